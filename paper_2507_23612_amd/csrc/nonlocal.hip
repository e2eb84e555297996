// Projector scatter of the nonlocal (KB) and Hubbard terms:
//
//   Y[s](x) += alpha * sum_j phi_j(x) Q[j][s]
//
// (Sec. II.A potential section: V_U psi = sum phi_m' U/2 (delta - 2D) <phi_m|psi>;
// Sec. II.B: implemented like the nonlocal projectors).  Each point owns its
// output (no atomics, deterministic).
//
// Real blocks: the grid is cut into bricks of 64 consecutive points; each
// brick stores the dense tile Phi_b over the functions touching it (padded
// to a multiple of 4).  A workgroup updates one brick for 64 states as a
// small GEMM on the matrix cores,
//   Y_b^T (64 states x 64 pts) += alpha Q^T (64 x nj) Phi_b (nj x 64),
// so every table value is read once per 64 states.
// Complex blocks: a thread reads the point's list of (function, value) pairs
// once and applies it to S states.
#include "common.h"

namespace hcu {

template <typename T, int S>
__global__ __launch_bounds__(256) void k_nl_scatter(T* __restrict__ Y, int64_t ld, int ncol,
                                                    const int* __restrict__ csr_ptr,
                                                    const int* __restrict__ csr_col,
                                                    const T* __restrict__ csr_val, const T* __restrict__ Qt,
                                                    int ldq, typename real_of<T>::type alpha, int64_t nd) {
  const int s0 = blockIdx.x * S;
  const int64_t p = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
  if (p >= nd) return;
  const int e0 = csr_ptr[p], e1 = csr_ptr[p + 1];
  if (e0 == e1) return;
  const int nh = min(S, ncol - s0);
  T acc[S];
  for (int s = 0; s < S; ++s) acc[s] = T(0);
  const T* __restrict__ Q0 = Qt + s0;
  for (int e = e0; e < e1; ++e) {
    const T v = csr_val[e];
    const T* __restrict__ q = Q0 + (int64_t)csr_col[e] * ldq;
    if (nh == S) {
      for (int s = 0; s < S; ++s) acc[s] += v * q[s];
    } else {
      for (int s = 0; s < S; ++s)
        if (s < nh) acc[s] += v * q[s];
    }
  }
  T* __restrict__ Yp = Y + (int64_t)s0 * ld + p;
  for (int s = 0; s < S; ++s)
    if (s < nh) Yp[(int64_t)s * ld] += alpha * acc[s];
}

// Workgroup: 4 waves x 16 states = 64 states, one brick of 64 points.
// Wave w owns states s0 + 16 w .. + 16 and computes
// D'(16 s x 16 p) += A'(16 s x 4 j) B'(4 j x 16 p) for the brick's 4 point
// tiles, with A' = alpha Q^T (lane: s = l%16, j = l/16) and
// B' = Phi (j = l/16, p = l%16); D' starts from Y and is written back.
template <typename T>
__global__ __launch_bounds__(256) void k_nl_brick(T* __restrict__ Y, int64_t ld, int ncol,
                                                  const int64_t* __restrict__ boff, const int* __restrict__ bnj,
                                                  const int* __restrict__ bj, const T* __restrict__ bval,
                                                  const T* __restrict__ Qt, int ldq, T alpha, int64_t nd, int nst) {
  using V = typename Mf<T>::V;
  // 1-D grid, logical order: state tile fastest, then brick; XCD-contiguous
  // so the state tiles of a brick share its table tile in one L2
  const unsigned lw = xcd_linear();
  const int b = lw / nst;
  const int st_ = lw % nst;
  const int64_t jo = boff[b];
  const int nj4 = (bnj[b] + 3) & ~3;
  if (nj4 == 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int s0 = st_ * 64 + wave * 16;
  const int sa = s0 + (lane & 15);
  const bool sa_ok = sa < ncol;
  const int64_t p0 = (int64_t)b * kBrick;
  const T* __restrict__ vb = bval + jo * kBrick;
  V acc[4];
  for (int pt = 0; pt < 4; ++pt)
    for (int q = 0; q < 4; ++q) {
      const int s = s0 + Mf<T>::row(lane, q);
      const int64_t p = p0 + pt * 16 + (lane & 15);
      acc[pt][q] = (s < ncol && p < nd) ? Y[(int64_t)s * ld + p] : T(0);
    }
  for (int jj = 0; jj < nj4; jj += 4) {
    const int jl = jj + (lane >> 4);
    const int jg = bj[jo + jl];
    const T a = (sa_ok && jg >= 0) ? alpha * Qt[(int64_t)jg * ldq + sa] : T(0);
    for (int pt = 0; pt < 4; ++pt) {
      const T bb = vb[(int64_t)jl * kBrick + pt * 16 + (lane & 15)];
      acc[pt] = Mf<T>::mfma(a, bb, acc[pt]);
    }
  }
  for (int pt = 0; pt < 4; ++pt)
    for (int q = 0; q < 4; ++q) {
      const int s = s0 + Mf<T>::row(lane, q);
      const int64_t p = p0 + pt * 16 + (lane & 15);
      if (s < ncol && p < nd) Y[(int64_t)s * ld + p] = acc[pt][q];
    }
}

template <typename T>
void launch_nl_scatter(const Ctx& c, int ik, T* Y, int64_t ld, int ncol, const T* Qt, double alpha,
                       hipStream_t st) {
  if (c.nproj == 0) return;
  if constexpr (sizeof(T) == sizeof(typename real_of<T>::type)) {
    const int nbrick = (int)c.boff.size() - 1;
    const int nst = (ncol + 63) / 64;
    k_nl_brick<T><<<(unsigned)nbrick * nst, 256, 0, st>>>(Y, ld, ncol, c.d_boff, c.d_bnj, c.d_bj,
                                                           (const T*)c.d_bval[ik], Qt, c.p.ns, (T)alpha, c.nd, nst);
    return;
  }
  constexpr int S = 8;
  dim3 grid((ncol + S - 1) / S, (unsigned)((c.nd + 255) / 256));
  k_nl_scatter<T, S><<<grid, 256, 0, st>>>(Y, ld, ncol, c.d_csr_ptr, c.d_csr_col, (const T*)c.d_csrv[ik], Qt,
                                            c.p.ns, (typename real_of<T>::type)alpha, c.nd);
}


template void launch_nl_scatter<double>(const Ctx&, int, double*, int64_t, int, const double*, double, hipStream_t);
template void launch_nl_scatter<float>(const Ctx&, int, float*, int64_t, int, const float*, double, hipStream_t);
template void launch_nl_scatter<cplx<double>>(const Ctx&, int, cplx<double>*, int64_t, int, const cplx<double>*,
                                              double, hipStream_t);
template void launch_nl_scatter<cplx<float>>(const Ctx&, int, cplx<float>*, int64_t, int, const cplx<float>*,
                                             double, hipStream_t);

}  // namespace hcu
