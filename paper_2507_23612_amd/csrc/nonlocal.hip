// Projector scatter of the nonlocal (KB) and Hubbard terms:
//
//   Y[s](x) += alpha * sum_j phi_j(x) Q[j][s]
//
// (Sec. II.A potential section: V_U psi = sum phi_m' U/2 (delta - 2D) <phi_m|psi>;
// Sec. II.B: implemented like the nonlocal projectors).  Each point owns its
// output (no atomics, deterministic).
//
// The grid is cut into bricks of 64 consecutive points; each brick stores
// the dense tile Phi_b over the functions touching it (padded to a multiple
// of 4).  A workgroup updates one brick for 64 states as a small GEMM on the
// matrix cores,
//   Y_b^T (64 states x 64 pts) += alpha Q^T (64 x nj) Phi_b (nj x 64),
// so every table value is read once per 64 states (complex blocks: four real
// products per step).
#include "common.h"

namespace hcu {

// Workgroup: 4 waves x 16 states = 64 states, one brick of 64 points.
// Wave w owns states s0 + 16 w .. + 16 and computes
// D'(16 s x 16 p) += A'(16 s x 4 j) B'(4 j x 16 p) for the brick's 4 point
// tiles, with A' = alpha Q^T (lane: s = l%16, j = l/16) and
// B' = Phi (j = l/16, p = l%16); D' starts from Y and is written back.
// groups of 4 functions per step; with two groups the kernel fits five
// waves per SIMD, which hides the load latency better than deeper batches
constexpr int kScatterU = 2;

template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_nl_brick(T* __restrict__ Y, int64_t ld, int ncol,
                                                  const int64_t* __restrict__ boff, const int* __restrict__ bnj,
                                                  const int* __restrict__ bj, const T* __restrict__ bval,
                                                  const T* __restrict__ Qt, int ldq, T alpha, int64_t nd, int nst,
                                                  const BrickGeo geo) {
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
  const int64_t p0 = geo.base(b);   // local index pt*16 + lane%16 at p0 + geo.off(...)
  const T* __restrict__ vb = bval + jo * kBrick;
  V acc[4];
  for (int pt = 0; pt < 4; ++pt)
    for (int q = 0; q < 4; ++q) {
      const int s = s0 + Mf<T>::row(lane, q);
      const int64_t p = p0 + geo.off(pt * 16 + (lane & 15));
      acc[pt][q] = (s < ncol && p < nd) ? Y[(int64_t)s * ld + p] : T(0);
    }
  // The brick's function indices are read 64 at a time (one per lane) and
  // handed to the lanes that need them by cross-lane reads, so the loop has
  // no index -> coefficient load chain; each step issues all its loads
  // (4 kScatterU functions) before the matrix-core ops.
  int bjl = -1;
  for (int jj = 0; jj < nj4; jj += 4 * kScatterU) {
    if ((jj & 63) == 0) {
      const int e = jj + lane;
      bjl = e < nj4 ? bj[jo + e] : -1;
    }
    T a[kScatterU], bb[kScatterU][4];
    for (int u = 0; u < kScatterU; ++u) {
      const int jl = jj + 4 * u + (lane >> 4);
      a[u] = T(0);
      for (int pt = 0; pt < 4; ++pt) bb[u][pt] = T(0);
      if (jj + 4 * u < nj4) {   // wave-uniform
        const int jg = __shfl(bjl, jl & 63);
        if (sa_ok && jg >= 0) a[u] = alpha * Qt[(int64_t)jg * ldq + sa];
        for (int pt = 0; pt < 4; ++pt) bb[u][pt] = vb[(int64_t)jl * kBrick + pt * 16 + (lane & 15)];
      }
    }
    for (int u = 0; u < kScatterU; ++u) {
      if (jj + 4 * u >= nj4) break;
      for (int pt = 0; pt < 4; ++pt) acc[pt] = Mf<T>::mfma(a[u], bb[u][pt], acc[pt]);
    }
  }
  for (int pt = 0; pt < 4; ++pt)
    for (int q = 0; q < 4; ++q) {
      const int s = s0 + Mf<T>::row(lane, q);
      const int64_t p = p0 + geo.off(pt * 16 + (lane & 15));
      if (s < ncol && p < nd) Y[(int64_t)s * ld + p] = acc[pt][q];
    }
}

// Complex (Bloch) blocks: the same brick GEMM in four real products,
//   Re Y += Re(aQ) Re Phi - Im(aQ) Im Phi,  Im Y += Re(aQ) Im Phi + Im(aQ) Re Phi.
template <typename R>
__global__ __launch_bounds__(256) void k_nl_brick_c(cplx<R>* __restrict__ Y, int64_t ld, int ncol,
                                                    const int64_t* __restrict__ boff, const int* __restrict__ bnj,
                                                    const int* __restrict__ bj, const cplx<R>* __restrict__ bval,
                                                    const cplx<R>* __restrict__ Qt, int ldq, R alpha, int64_t nd,
                                                    int nst, const BrickGeo geo) {
  using V = typename Mf<R>::V;
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
  const int64_t p0 = geo.base(b);   // local index pt*16 + lane%16 at p0 + geo.off(...)
  const cplx<R>* __restrict__ vb = bval + jo * kBrick;
  // Loads from clamped in-range addresses, zeroed by selection afterwards:
  // a conditional load becomes a branch that waits for every outstanding
  // load before the next one issues.
  V ar[4], ai[4];
  {
    cplx<R> yv[4][4];
    for (int pt = 0; pt < 4; ++pt)
      for (int q = 0; q < 4; ++q) {
        const int s = min(s0 + Mf<R>::row(lane, q), ncol - 1);
        const int64_t p = min(p0 + geo.off(pt * 16 + (lane & 15)), nd - 1);
        yv[pt][q] = Y[(int64_t)s * ld + p];
      }
    for (int pt = 0; pt < 4; ++pt)
      for (int q = 0; q < 4; ++q) {
        const bool in = s0 + Mf<R>::row(lane, q) < ncol && p0 + geo.off(pt * 16 + (lane & 15)) < nd;
        ar[pt][q] = in ? yv[pt][q].re : R(0);
        ai[pt][q] = in ? yv[pt][q].im : R(0);
      }
  }
  // function indices 64 at a time, passed between lanes (the index array has
  // a 64-entry tail, so the unguarded load stays inside it); Q is zeroed at
  // its use, so a step's loads go out together
  const int sac = sa_ok ? sa : ncol - 1;
  int bjl = -1;
  for (int jj = 0; jj < nj4; jj += 4) {
    if ((jj & 63) == 0) {
      const int v = bj[jo + jj + lane];
      bjl = jj + lane < nj4 ? v : -1;
    }
    const int jl = jj + (lane >> 4);
    const int jg = __shfl(bjl, jl & 63);
    const cplx<R> qraw = Qt[(int64_t)(jg >= 0 ? jg : 0) * ldq + sac];
    const bool qok = sa_ok && jg >= 0;
    const R qr = qok ? alpha * qraw.re : R(0), qi = qok ? alpha * qraw.im : R(0);
    cplx<R> f[4];
    for (int pt = 0; pt < 4; ++pt) f[pt] = vb[(int64_t)jl * kBrick + pt * 16 + (lane & 15)];
    // independent accumulators between dependent matrix-core ops
    for (int pt = 0; pt < 4; ++pt) {
      ar[pt] = Mf<R>::mfma(qr, f[pt].re, ar[pt]);
      ai[pt] = Mf<R>::mfma(qr, f[pt].im, ai[pt]);
    }
    for (int pt = 0; pt < 4; ++pt) {
      ar[pt] = Mf<R>::mfma(-qi, f[pt].im, ar[pt]);
      ai[pt] = Mf<R>::mfma(qi, f[pt].re, ai[pt]);
    }
  }
  for (int pt = 0; pt < 4; ++pt)
    for (int q = 0; q < 4; ++q) {
      const int s = s0 + Mf<R>::row(lane, q);
      const int64_t p = p0 + geo.off(pt * 16 + (lane & 15));
      if (s < ncol && p < nd) Y[(int64_t)s * ld + p] = cplx<R>(ar[pt][q], ai[pt][q]);
    }
}

template <typename T>
void launch_nl_scatter(const Ctx& c, int ik, T* Y, int64_t ld, int ncol, const T* Qt, double alpha,
                       hipStream_t st) {
  if (c.nproj == 0) return;
  if constexpr (sizeof(T) == sizeof(typename real_of<T>::type)) {
    const int nbrick = (int)c.boff.size() - 1;
    const int nst = (ncol + 63) / 64;
    launch_k(k_nl_brick<T>, (unsigned)nbrick * nst, 256, 0, st, Y, ld, ncol, c.d_boff, c.d_bnj, c.d_bj,
             (const T*)c.d_bval[ik], Qt, c.p.ns, (T)alpha, c.nd, nst, c.geo);
    return;
  }
  else {
    using R = typename real_of<T>::type;
    const int nbrick = (int)c.boff.size() - 1;
    const int nst = (ncol + 63) / 64;
    launch_k(k_nl_brick_c<R>, (unsigned)nbrick * nst, 256, 0, st, Y, ld, ncol, c.d_boff, c.d_bnj, c.d_bj,
             (const T*)c.d_bval[ik], Qt, c.p.ns, (R)alpha, c.nd, nst, c.geo);
    return;
  }
}


template void launch_nl_scatter<double>(const Ctx&, int, double*, int64_t, int, const double*, double, hipStream_t);
template void launch_nl_scatter<float>(const Ctx&, int, float*, int64_t, int, const float*, double, hipStream_t);
template void launch_nl_scatter<cplx<double>>(const Ctx&, int, cplx<double>*, int64_t, int, const cplx<double>*,
                                              double, hipStream_t);
template void launch_nl_scatter<cplx<float>>(const Ctx&, int, cplx<float>*, int64_t, int, const cplx<float>*,
                                             double, hipStream_t);

}  // namespace hcu
