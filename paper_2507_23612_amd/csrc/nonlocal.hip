// Projector scatter of the nonlocal (KB) and Hubbard terms:
//
//   Y[s](x) += alpha * sum_j phi_j(x) Q[j][s]
//
// (Sec. II.A potential section: V_U psi = sum phi_m' U/2 (delta - 2D) <phi_m|psi>;
// Sec. II.B: implemented like the nonlocal projectors).  Each point owns its
// output (no atomics, deterministic): a thread reads the point's list of
// (function, value) pairs once and applies it to S states, so the per-point
// table is read once per S states; Q rows are contiguous in s.
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

template <typename T>
void launch_nl_scatter(const Ctx& c, int ik, T* Y, int64_t ld, int ncol, const T* Qt, double alpha,
                       hipStream_t st) {
  if (c.nproj == 0) return;
  constexpr int S = sizeof(T) > 8 ? 8 : 16;
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
