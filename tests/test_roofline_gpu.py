"""The streaming reference kernels behind the measured HBM ceiling and the
byte-counter calibration (cg_stream_probe): the copy kernel reproduces its
source exactly and the write kernel fills its buffer, for every grid/block
shape of the sweep and both cache policies (the rates they report are only
meaningful if they move the bytes they claim); the read kernel leaves its
output alone; bad arguments are refused."""
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_copy_and_write_kernels_move_every_byte():
    from paper_2407_10914_amd import roofline

    n = (64 << 20) // 4 + 4 * 37  # 64 MiB and a ragged tail of float4s
    src = torch.arange(n, dtype=torch.float32, device="cuda")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for nt in (False, True):
        for grid, block in ((cus, 256), (8 * cus, 512), (64 * cus, 1024), (7, 64)):
            dst = torch.full_like(src, -1.0)
            ms = roofline.probe("copy", src, dst, n * 4, grid, block, nt, reps=1)
            assert ms > 0.0
            assert torch.equal(dst, src), (nt, grid, block)
            out = torch.zeros_like(src)
            roofline.probe("write", src, out, n * 4, grid, block, nt, reps=1)
            assert torch.all(out == 1.0), (nt, grid, block)
            keep = torch.full((4,), 7.0, device="cuda")
            roofline.probe("read", src, keep, n * 4, grid, block, nt, reps=1)
            assert torch.all(keep == 7.0)


def test_probe_refuses_bad_arguments():
    from paper_2407_10914_amd import roofline
    from paper_2407_10914_amd.lib import CgError

    a = torch.zeros(1024, dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    for kind, nbytes, grid, block in (("copy", 4096, 0, 256), ("copy", 4096, 8, 96), ("copy", 4100, 8, 256),
                                      ("copy", 8, 8, 256)):
        with pytest.raises(CgError):
            roofline.probe(kind, a, b, nbytes, grid, block, False, reps=1)


def test_stream_ceiling_on_a_small_buffer():
    from paper_2407_10914_amd import roofline

    best, recs = roofline.stream_ceiling(gib=0.25, reps=2, grids=[256, 2048], blocks=(256,))
    assert set(best) == {"read", "write", "copy"}
    assert len(recs) == 3 * 2 * 2
    for r in recs:
        assert 0.0 < r["gbs"] < 12000.0, r
