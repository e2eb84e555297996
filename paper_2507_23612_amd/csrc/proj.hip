// Projections of a block of states onto the atom-centred functions
// (Sec. II.B: the integrals of every atom's functions, as for nonlocal
// projectors):
//
//   P[s][j] = dV * sum_x conj(phi_j(x)) y_s(x)                 (trapezoid rule)
//   Q[j][s] = sum_m' C_b[m][m'] P[s][j0+m']     (Q stored transposed for the scatter)
//
// with C_b = diag(gamma) for the KB channels and C_b = U (1/2 - D) for the
// Hubbard manifold (Eq. DerED).  The grid is cut into bricks of kPBrick
// consecutive points; each brick's functions form a dense value tile, and
// a workgroup computes the brick's partial projections for 64 states as a
// small GEMM on the matrix cores, reading every point-state value once.  The
// partials are summed per function in a fixed order (deterministic), then
// the coupling is applied.
#include "common.h"

#include <algorithm>

namespace hcu {

// ---------------------------------------------------------------- real blocks
// Stage 1, one workgroup per (projection brick of kPBrick points, 64 states),
// wave w owning 16 states:
//   part[pdest[slot]][s] = sum_{p in brick} Phi_b[slot][p] y_s(p)
// as D(16 slots x 16 s) += A(16 slots x 4) B(4 x 16 s) on the matrix cores.
// The contraction runs over the brick's points in the order
// p = piece*64 + 16 q + kk, with q = l/16 the depth index of lane l and kk
// the step: lane l then needs 16 consecutive points of its state row (one
// 128-byte run for FP64) and 16 consecutive table values (the table is stored
// in that order), so both operands are read with wide contiguous loads.
// Every point-state value is read once per launch.
template <typename T>
__device__ __forceinline__ void load16(const T* __restrict__ p, bool vec, int64_t n_ok, T* out) {
  if (vec && n_ok >= 16) {
    if constexpr (sizeof(T) == 8) {
      using D2 = double __attribute__((ext_vector_type(2)));
      const D2* v = reinterpret_cast<const D2*>(p);
      for (int i = 0; i < 8; ++i) {
        const D2 x = v[i];
        out[2 * i] = x[0];
        out[2 * i + 1] = x[1];
      }
    } else {
      using F4 = float __attribute__((ext_vector_type(4)));
      const F4* v = reinterpret_cast<const F4*>(p);
      for (int i = 0; i < 4; ++i) {
        const F4 x = v[i];
        out[4 * i] = x[0];
        out[4 * i + 1] = x[1];
        out[4 * i + 2] = x[2];
        out[4 * i + 3] = x[3];
      }
    }
  } else {
    for (int i = 0; i < 16; ++i) out[i] = i < n_ok ? p[i] : T(0);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_proj_brick(const T* __restrict__ Y, int64_t ld, int ncol,
                                                    const int64_t* __restrict__ pboff, const int* __restrict__ pbnj,
                                                    const T* __restrict__ pbval, const int64_t* __restrict__ pdest,
                                                    T* __restrict__ part, int ldp, int64_t nd, int nst, int vec) {
  using V = typename Mf<T>::V;
  const unsigned lw = xcd_linear();   // 1-D grid: state tile fastest, then brick
  const int b = lw / nst;
  const int st_ = lw % nst;
  const int nj = pbnj[b];
  if (nj == 0) return;
  const int64_t jo = pboff[b];
  const int ntile = (nj + 15) / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int s0 = st_ * 64 + wave * 16;
  if (s0 >= ncol) return;
  const int sb = s0 + (lane & 15);
  const int q = lane >> 4;
  const int64_t p0 = (int64_t)b * kPBrick;
  const T* __restrict__ Ys = Y + (int64_t)min(sb, ncol - 1) * ld;
  const bool vec_ok = vec != 0;
  if constexpr (sizeof(T) == 8) {
    // FP64: up to four slot tiles per sweep, one accumulator each (the
    // register budget keeps three waves per SIMD)
    for (int jg = 0; jg < ntile; jg += 4) {
      V acc[4];
      for (int t = 0; t < 4; ++t)
        for (int r = 0; r < 4; ++r) acc[t][r] = T(0);
      for (int piece = 0; piece < kPBrick / 64; ++piece) {
        const int64_t pb = p0 + piece * 64 + 16 * q;
        T bk[16];
        const int64_t n_ok = sb < ncol ? max((int64_t)0, min((int64_t)16, nd - pb)) : 0;
        load16<T>(Ys + pb, vec_ok, n_ok, bk);
        for (int t = 0; t < 4; ++t) {
          if (jg + t >= ntile) break;   // wave-uniform
          T a[16];
          load16<T>(pbval + ((((jo / 16 + jg + t) * (kPBrick / 64) + piece) * 64 + lane) * 16), true, 16, a);
          for (int kk = 0; kk < 16; ++kk) acc[t] = Mf<T>::mfma(a[kk], bk[kk], acc[t]);
        }
      }
      for (int t = 0; t < 4; ++t) {
        if (jg + t >= ntile) break;
        for (int r = 0; r < 4; ++r) {
          const int j = (jg + t) * 16 + Mf<T>::row(lane, r);
          if (j < nj && sb < ncol) part[pdest[jo + j] * ldp + sb] = acc[t][r];
        }
      }
    }
  } else {
    // two slot tiles per sweep; each tile keeps two accumulators (even and odd
    // depth steps) so that consecutive matrix-core ops are independent
    for (int jg = 0; jg < ntile; jg += 2) {
      const bool two = jg + 1 < ntile;   // wave-uniform
      V acc[2][2];
      for (int t = 0; t < 2; ++t)
        for (int h = 0; h < 2; ++h)
          for (int r = 0; r < 4; ++r) acc[t][h][r] = T(0);
      for (int piece = 0; piece < kPBrick / 64; ++piece) {
        const int64_t pb = p0 + piece * 64 + 16 * q;
        T bk[16], a0[16], a1[16];
        const int64_t n_ok = sb < ncol ? max((int64_t)0, min((int64_t)16, nd - pb)) : 0;
        load16<T>(Ys + pb, vec_ok, n_ok, bk);
        load16<T>(pbval + ((((jo / 16 + jg) * (kPBrick / 64) + piece) * 64 + lane) * 16), true, 16, a0);
        if (two) {
          load16<T>(pbval + ((((jo / 16 + jg + 1) * (kPBrick / 64) + piece) * 64 + lane) * 16), true, 16, a1);
          for (int kk = 0; kk < 16; ++kk) {
            acc[0][kk & 1] = Mf<T>::mfma(a0[kk], bk[kk], acc[0][kk & 1]);
            acc[1][kk & 1] = Mf<T>::mfma(a1[kk], bk[kk], acc[1][kk & 1]);
          }
        } else {
          for (int kk = 0; kk < 16; ++kk) acc[0][kk & 1] = Mf<T>::mfma(a0[kk], bk[kk], acc[0][kk & 1]);
        }
      }
      for (int t = 0; t < (two ? 2 : 1); ++t)
        for (int r = 0; r < 4; ++r) {
          const int j = (jg + t) * 16 + Mf<T>::row(lane, r);
          if (j < nj && sb < ncol) part[pdest[jo + j] * ldp + sb] = acc[t][0][r] + acc[t][1][r];
        }
    }
  }
}

// Complex (Bloch) blocks: the same brick GEMM with P = Phi^H y, as four
// real matrix-core products per step,
//   Re P += Re Phi Re y + Im Phi Im y,   Im P += Re Phi Im y - Im Phi Re y.
template <typename R>
__device__ __forceinline__ void load16c(const cplx<R>* __restrict__ p, bool vec, int64_t n_ok, R* re, R* im) {
  if (vec && n_ok >= 16) {
    if constexpr (sizeof(R) == 8) {
      using D2 = double __attribute__((ext_vector_type(2)));
      const D2* v = reinterpret_cast<const D2*>(p);
      for (int i = 0; i < 16; ++i) {
        const D2 x = v[i];
        re[i] = x[0];
        im[i] = x[1];
      }
    } else {
      using F4 = float __attribute__((ext_vector_type(4)));
      const F4* v = reinterpret_cast<const F4*>(p);
      for (int i = 0; i < 8; ++i) {
        const F4 x = v[i];
        re[2 * i] = x[0];
        im[2 * i] = x[1];
        re[2 * i + 1] = x[2];
        im[2 * i + 1] = x[3];
      }
    }
  } else {
    for (int i = 0; i < 16; ++i) {
      const cplx<R> x = i < n_ok ? p[i] : cplx<R>();
      re[i] = x.re;
      im[i] = x.im;
    }
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_proj_brick_c(const cplx<R>* __restrict__ Y, int64_t ld, int ncol,
                                                      const int64_t* __restrict__ pboff,
                                                      const int* __restrict__ pbnj,
                                                      const cplx<R>* __restrict__ pbval,
                                                      const int64_t* __restrict__ pdest, cplx<R>* __restrict__ part,
                                                      int ldp, int64_t nd, int nst, int vec) {
  using V = typename Mf<R>::V;
  const unsigned lw = xcd_linear();
  const int b = lw / nst;
  const int st_ = lw % nst;
  const int nj = pbnj[b];
  if (nj == 0) return;
  const int64_t jo = pboff[b];
  const int ntile = (nj + 15) / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int s0 = st_ * 64 + wave * 16;
  if (s0 >= ncol) return;
  const int sb = s0 + (lane & 15);
  const int q = lane >> 4;
  const int64_t p0 = (int64_t)b * kPBrick;
  const cplx<R>* __restrict__ Ys = Y + (int64_t)min(sb, ncol - 1) * ld;
  const bool vec_ok = vec != 0;
  // one slot tile per sweep with four independent accumulators
  // (Re Phi Re y, Im Phi Im y, Re Phi Im y, Im Phi Re y)
  for (int jt = 0; jt < ntile; ++jt) {
    V c0, c1, c2, c3;
    for (int r = 0; r < 4; ++r) c0[r] = c1[r] = c2[r] = c3[r] = R(0);
    for (int piece = 0; piece < kPBrick / 64; ++piece) {
      const int64_t pb = p0 + piece * 64 + 16 * q;
      R yr[16], yi[16], fr[16], fi[16];
      const int64_t n_ok = sb < ncol ? max((int64_t)0, min((int64_t)16, nd - pb)) : 0;
      load16c<R>(Ys + pb, vec_ok, n_ok, yr, yi);
      load16c<R>(pbval + ((((jo / 16 + jt) * (kPBrick / 64) + piece) * 64 + lane) * 16), true, 16, fr, fi);
      for (int kk = 0; kk < 16; ++kk) {
        c0 = Mf<R>::mfma(fr[kk], yr[kk], c0);
        c1 = Mf<R>::mfma(fi[kk], yi[kk], c1);
        c2 = Mf<R>::mfma(fr[kk], yi[kk], c2);
        c3 = Mf<R>::mfma(fi[kk], yr[kk], c3);
      }
    }
    for (int r = 0; r < 4; ++r) {
      const int j = jt * 16 + Mf<R>::row(lane, r);
      if (j < nj && sb < ncol) part[pdest[jo + j] * ldp + sb] = cplx<R>(c0[r] + c1[r], c2[r] - c3[r]);
    }
  }
}

// Stage 2: P[s][j] = dV * sum of rows jrow[j] .. jrow[j+1] of part (fixed
// order).  One workgroup per (j, 64 states); its 16 waves take every 16th
// row and are combined in a fixed order.
template <typename T>
__global__ __launch_bounds__(1024) void k_slot_sum(const T* __restrict__ part, int ldp, int ncol,
                                                   const int64_t* __restrict__ jrow, T* __restrict__ P, int nproj,
                                                   double dv) {
  using RT = typename real_of<T>::type;
  __shared__ __attribute__((aligned(16))) unsigned char red_raw[16 * 64 * sizeof(T)];
  T(*red)[64] = reinterpret_cast<T(*)[64]>(red_raw);
  const int j = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int s = blockIdx.x * 64 + lane;
  T x0 = T(0), x1 = T(0);
  if (s < ncol) {
    const int64_t r1 = jrow[j + 1];
    int64_t r = jrow[j] + wave;
    for (; r + 16 < r1; r += 32) {
      x0 += part[r * ldp + s];
      x1 += part[(r + 16) * ldp + s];
    }
    if (r < r1) x0 += part[r * ldp + s];
  }
  red[wave][lane] = x0 + x1;
  __syncthreads();
  if (wave == 0 && s < ncol) {
    T x = T(0);
    for (int w = 0; w < 16; ++w) x += red[w][lane];
    P[(int64_t)s * nproj + j] = (RT)dv * x;
  }
}

// Q[j0+m][s] = sum_m' C_b[m][m'] P[s][j0+m'], one thread per (block, state).
template <typename T>
__global__ void k_couple(const T* __restrict__ P, const BlockDesc* __restrict__ blocks, int ncol,
                         const double* __restrict__ coup, T* __restrict__ Q, int nproj, int ldq) {
  const BlockDesc& b = blocks[blockIdx.y];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ncol) return;
  using RT = typename real_of<T>::type;
  T pv[kMaxNm];
  for (int m = 0; m < b.nm; ++m) pv[m] = P[(int64_t)s * nproj + b.j0 + m];
  const double* cb = coup + b.coup_off;
  for (int m = 0; m < b.nm; ++m) {
    T qv = T(0);
    for (int mp = 0; mp < b.nm; ++mp) qv += (RT)cb[m * b.nm + mp] * pv[mp];
    Q[(int64_t)(b.j0 + m) * ldq + s] = qv;
  }
}

size_t project_partial_elems(const Ctx& c) {
  if (c.pboff.empty()) return 0;
  return (size_t)c.pboff.back() * c.p.ns;
}

template <typename T>
void launch_project_brick(const Ctx& c, int ik, const T* Y, int ncol, int64_t ld, const double* coup, T* P, T* Q,
                          hipStream_t st) {
  if (c.nproj == 0) return;
  T* part = reinterpret_cast<T*>(c.d_ppart);
  const int npb = (int)c.pboff.size() - 1;
  const int nst = (ncol + 63) / 64;
  // wide loads of the state rows need 16-byte aligned rows
  const int vec = ((uintptr_t)Y % 16 == 0 && (ld * (int64_t)sizeof(T)) % 16 == 0) ? 1 : 0;
  if constexpr (sizeof(T) == sizeof(typename real_of<T>::type))
    launch_k(k_proj_brick<T>, (unsigned)npb * nst, 256, 0, st, Y, ld, ncol, c.d_pboff, c.d_pbnj,
             (const T*)c.d_pbval[ik], c.d_pdest, part, c.p.ns, c.nd, nst, vec);
  else
    launch_k(k_proj_brick_c<typename real_of<T>::type>, (unsigned)npb * nst, 256, 0, st, Y, ld, ncol, c.d_pboff,
             c.d_pbnj, (const T*)c.d_pbval[ik], c.d_pdest, part, c.p.ns, c.nd, nst, vec);
  dim3 g2((ncol + 63) / 64, c.nproj);
  launch_k(k_slot_sum<T>, g2, 1024, 0, st, part, c.p.ns, ncol, c.d_jrow, P, c.nproj, c.dv);
  dim3 g3((ncol + 63) / 64, (unsigned)c.blocks.size());
  launch_k(k_couple<T>, g3, 64, 0, st, P, c.d_blocks, ncol, coup, Q, c.nproj, c.p.ns);
}

template void launch_project_brick<double>(const Ctx&, int, const double*, int, int64_t, const double*, double*,
                                           double*, hipStream_t);
template void launch_project_brick<float>(const Ctx&, int, const float*, int, int64_t, const double*, float*,
                                          float*, hipStream_t);
template void launch_project_brick<cplx<double>>(const Ctx&, int, const cplx<double>*, int, int64_t, const double*,
                                                 cplx<double>*, cplx<double>*, hipStream_t);
template void launch_project_brick<cplx<float>>(const Ctx&, int, const cplx<float>*, int, int64_t, const double*,
                                                cplx<float>*, cplx<float>*, hipStream_t);

}  // namespace hcu
