// Compile-time lattice tables for the device code.
//
// D3Q19: velocity set and weights of Appendix A, Eqs. (A.1)-(A.2).
// D2Q9: the in-plane directions of that set, kept in the same order, with the
// D2Q9 weights 4/9, 1/9, 1/36.
// The MRT matrix of Eq. (A.3) is generated from the polynomial that defines
// each moment of Eq. (3) (two rows of the printed matrix are garbled), and
// M^-1 = M^T diag(1/|row|^2) because the rows are orthogonal.
//
// Everything here is constexpr and is only ever indexed with compile-time
// constants (see unroll<>), so it folds into immediates in the kernels.
#pragma once

#include <type_traits>
#include <utility>

namespace cg {

template <int N, class F>
__host__ __device__ __forceinline__ void unroll(F&& f) {
  if constexpr (N > 0) {
    unroll<N - 1>(f);
    f(std::integral_constant<int, N - 1>{});
  }
}

template <int D>
struct Lat;

template <>
struct Lat<3> {
  static constexpr int Q = 19;
  static constexpr int D = 3;
  __host__ __device__ static constexpr int e(int i, int a) {
    // columns of Eq. (A.1)
    constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    constexpr int ey[19] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1};
    constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
    return a == 0 ? ex[i] : (a == 1 ? ey[i] : ez[i]);
  }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
  }
};

template <>
struct Lat<2> {
  static constexpr int Q = 9;
  static constexpr int D = 2;
  __host__ __device__ static constexpr int e(int i, int a) {
    constexpr int ex[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
    constexpr int ey[9] = {0, 0, 0, 1, -1, 1, 1, -1, -1};
    return a == 0 ? ex[i] : (a == 1 ? ey[i] : 0);
  }
  __host__ __device__ static constexpr double w(int i) {
    return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
  }
};

template <int D>
__host__ __device__ constexpr int opp(int i) {
  for (int j = 0; j < Lat<D>::Q; ++j)
    if (Lat<D>::e(j, 0) == -Lat<D>::e(i, 0) && Lat<D>::e(j, 1) == -Lat<D>::e(i, 1) &&
        Lat<D>::e(j, 2) == -Lat<D>::e(i, 2))
      return j;
  return -1;
}

// index of the direction with velocity (0, 0, +1): its pull source is x - e_z
constexpr int kDirZp = 5;

// Moment k of Eq. (3) evaluated at velocity (ex, ey, ez).
__host__ __device__ constexpr int moment_row(int k, int ex, int ey, int ez) {
  const int c2 = ex * ex + ey * ey + ez * ez;
  const int qx = 3 * ex * ex - c2;
  const int ww = ey * ey - ez * ez;
  switch (k) {
    case 0: return 1;
    case 1: return 19 * c2 - 30;
    case 2: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
    case 3: return ex;
    case 4: return (5 * c2 - 9) * ex;
    case 5: return ey;
    case 6: return (5 * c2 - 9) * ey;
    case 7: return ez;
    case 8: return (5 * c2 - 9) * ez;
    case 9: return qx;
    case 10: return (3 * c2 - 5) * qx;
    case 11: return ww;
    case 12: return (3 * c2 - 5) * ww;
    case 13: return ex * ey;
    case 14: return ey * ez;
    case 15: return ex * ez;
    case 16: return ex * ww;
    case 17: return ey * (ez * ez - ex * ex);
    default: return ez * (ex * ex - ey * ey);
  }
}

__host__ __device__ constexpr int Mkj(int k, int i) {
  return moment_row(k, Lat<3>::e(i, 0), Lat<3>::e(i, 1), Lat<3>::e(i, 2));
}

__host__ __device__ constexpr int Mnorm2(int k) {
  int s = 0;
  for (int i = 0; i < 19; ++i) s += Mkj(k, i) * Mkj(k, i);
  return s;
}

// (M^-1)_{ik} = M_{ki} / |row k|^2
__host__ __device__ constexpr double Minv(int i, int k) { return (double)Mkj(k, i) / (double)Mnorm2(k); }

// Relaxation-rate class of moment k in Eq. (4): 0 conserved, 1 S_nu
// (e, epsilon, the stress and pi moments), 2 S_q (q and m moments).
__host__ __device__ constexpr int rate_class(int k) {
  return (k == 0 || k == 3 || k == 5 || k == 7) ? 0 : ((k == 4 || k == 6 || k == 8 || k >= 16) ? 2 : 1);
}

}  // namespace cg
