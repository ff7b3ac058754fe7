// Once-per-run host setup (FP64): voxel classes, boundary sets along lattice
// links, the smoothed image and wall normal of Eqs. (25)-(26), the contact
// angle at each fluid boundary point, the sparse fluid-node index and the pull
// table.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cg_lbm.h"

namespace cg {

struct HostSetup {
  int dim = 3, Q = 19, nx = 0, ny = 0, nz = 0, V = 0;
  int per[3] = {0, 0, 0};
  int bc = 0;
  int N = 0;   // fluid nodes
  int Np = 0;  // padded stride
  int n_fb = 0, n_in = 0, n_out = 0;
  std::vector<int> node_vox;    // [N]
  std::vector<int> nbr;         // [(Q-1) * Np]
  // 16-bit form of nbr (see Nbr in step.hpp); empty when some offset does not fit
  std::vector<int16_t> nbr16;   // [(Q-1) * Np]
  std::vector<int> nbr_base;    // [(Q-1) * ntiles]
  int ntiles = 0;
  // 8-bit pull table per wave of 64 nodes (see Nbr in step.hpp); empty when
  // not used
  std::vector<uint32_t> nbr8;   // [Np/64][(Q-1+3)/4][64]
  std::vector<int> nbr8_head;   // [Np/64][Q-1]: the wave's base per direction
  long n8_waves = 0;            // waves of the 8-bit table whose offsets fit
  std::vector<unsigned> flags;  // [Np]
  std::vector<int> sb_vox;      // [nsb]
  std::vector<unsigned> sb_mask;
  std::vector<double> nw;       // [3 * Np]
  std::vector<double> cos_t, sin_t;  // [Np]
  std::vector<double> sb_fd;    // [nsb] fictitious-density phase -cos(theta), Eq. (24)
  std::vector<double> g3;       // smoothed image [V] (kept for diagnostics)
  // solid link neighbours of each fluid boundary point, i ascending:
  // fb_node[k] has links fb_off[k] .. fb_off[k+1]-1 to voxels fb_vox with weights fb_w
  std::vector<int> fb_node, fb_off, fb_vox;
  std::vector<double> fb_w;
  int s1_line = 0;
};

// Contact angle at every fluid boundary point from the global angle or the
// per-voxel field (w_i-weighted mean over the solid link neighbours): fills
// cos_t, sin_t and the FL_S1POS bit of flags for those nodes ([Np] each),
// and the fictitious-density phase of every solid boundary point from its
// own angle (sb_fd, [nsb]).  The arrays must have those sizes already.
// Returns CG_OK or CG_EINVAL with *err set.
int contact_angles(const HostSetup& S, double theta_deg, const double* theta_field_deg, std::vector<double>* cos_t,
                   std::vector<double>* sin_t, std::vector<unsigned>* flags, std::vector<double>* sb_fd,
                   std::string* err);

// pull_table: narrowest neighbour table to build (0 or 8, 16, 32; see
// cg_options).  Returns CG_OK or an error with *err set.
int build_setup(const cg_geometry& g, const cg_wetting& w, const cg_bc& bc, HostSetup* out, std::string* err,
                int pull_table = 0);

}  // namespace cg
