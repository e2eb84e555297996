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
#include <type_traits>

namespace hcu {

// ---------------------------------------------------------------- real blocks
// Stage 1, one workgroup per (projection brick of kPBrick points, 64 states),
// wave w owning 16 states:
//   part[pdest[slot]][s] = sum_{p in brick} Phi_b[slot][p] y_s(p)
// as D(16 slots x 16 s) += A(16 slots x 4) B(4 x 16 s) on the matrix cores.
// Operand order, for a group size G (points per lane and load group, a
// property of the context): at step t (0..15) of a 64-point piece, lane l
// (depth index q = l/16, column l%16) supplies the point
//   piece*64 + 4G*(t/G) + G*q + t%G,
// so each load instruction of a wave covers 4G consecutive points of each of
// its 16 state rows (4 lanes x G points), and the table, stored in the same
// order [tile][piece][t/G][lane][t%G], is read as one contiguous run per
// instruction.  G = 16 (a lane reads 16 consecutive points of its own row)
// touches 64 cache lines per instruction, and the vector-cache tag rate
// rather than HBM then limits FP64; G = 2 (16 bytes per lane in FP64) and
// G = 4 (FP32) cover each line with a quarter of the instructions.
// Every point-state value is read once per launch.

// G consecutive values at p (wide loads when vec: state rows and the table
// start 16-byte aligned and groups start at multiples of G)
template <typename T, int G>
__device__ __forceinline__ void ld_group(const T* __restrict__ p, bool vec, T* out) {
  constexpr int bytes = G * (int)sizeof(T);
  if (vec) {
    if constexpr (bytes % 16 == 0) {
      using F4 = float __attribute__((ext_vector_type(4)));
      F4 v[bytes / 16];
      for (int c = 0; c < bytes / 16; ++c) v[c] = reinterpret_cast<const F4*>(p)[c];
      __builtin_memcpy(out, v, bytes);
      return;
    } else if constexpr (bytes == 8) {
      using F2 = float __attribute__((ext_vector_type(2)));
      const F2 v = *reinterpret_cast<const F2*>(p);
      __builtin_memcpy(out, &v, bytes);
      return;
    }
  }
  for (int g = 0; g < G; ++g) out[g] = p[g];
}

// the 16 step operands of one piece: groups at row + i*stride + off; for
// state rows (stride 4G, off G q) n_here = points of the piece inside the
// grid, for the table (stride 64 G, off 0) n_here = 64
template <typename T, int G>
__device__ __forceinline__ void load_piece(const T* __restrict__ row, int stride, int off, int64_t n_here, bool vec,
                                           T* out) {
  if (n_here >= 64) {
    for (int i = 0; i < 16 / G; ++i) ld_group<T, G>(row + i * stride + off, vec, out + G * i);
  } else {
    for (int i = 0; i < 16 / G; ++i)
      for (int g = 0; g < G; ++g) {
        const int o = i * stride + off + g;
        out[G * i + g] = o < n_here ? row[o] : T();
      }
  }
}

template <typename T, int G>
__global__ __launch_bounds__(256) void k_proj_brick(const T* __restrict__ Y, int64_t ld, int ncol,
                                                    const int64_t* __restrict__ pboff, const int* __restrict__ pbnj,
                                                    const T* __restrict__ pbval, const int64_t* __restrict__ pdest,
                                                    T* __restrict__ part, int ldp, int64_t nd, int nst, int vec) {
  using V = typename Mf<T>::V;
  constexpr int P = kPBrick / 64;
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
  // rows of padding states repeat the last state (results never stored)
  const T* __restrict__ Ys = Y + (int64_t)min(sb, ncol - 1) * ld;
  const bool vec_ok = vec != 0;
  // table run of (tile, piece) for this lane
  auto trow = [&](int tile, int piece) {
    return pbval + (((jo / 16 + tile) * P + piece) * (16 / G)) * (64 * G) + lane * G;
  };
  if constexpr (sizeof(T) == 8) {
    // FP64: up to four slot tiles per sweep, one accumulator each (the
    // register budget keeps three waves per SIMD)
    for (int jg = 0; jg < ntile; jg += 4) {
      V acc[4];
      for (int t = 0; t < 4; ++t)
        for (int r = 0; r < 4; ++r) acc[t][r] = T(0);
      for (int piece = 0; piece < P; ++piece) {
        const int64_t pb = p0 + piece * 64;
        T bk[16];
        load_piece<T, G>(Ys + pb, 4 * G, G * q, nd - pb, vec_ok, bk);
        for (int t = 0; t < 4; ++t) {
          if (jg + t >= ntile) break;   // wave-uniform
          T a[16];
          load_piece<T, G>(trow(jg + t, piece), 64 * G, 0, 64, true, a);
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
      for (int piece = 0; piece < P; ++piece) {
        const int64_t pb = p0 + piece * 64;
        T bk[16], a0[16], a1[16];
        load_piece<T, G>(Ys + pb, 4 * G, G * q, nd - pb, vec_ok, bk);
        load_piece<T, G>(trow(jg, piece), 64 * G, 0, 64, true, a0);
        if (two) {
          load_piece<T, G>(trow(jg + 1, piece), 64 * G, 0, 64, true, a1);
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
template <typename R, int G>
__global__ __launch_bounds__(256) void k_proj_brick_c(const cplx<R>* __restrict__ Y, int64_t ld, int ncol,
                                                      const int64_t* __restrict__ pboff,
                                                      const int* __restrict__ pbnj,
                                                      const cplx<R>* __restrict__ pbval,
                                                      const int64_t* __restrict__ pdest, cplx<R>* __restrict__ part,
                                                      int ldp, int64_t nd, int nst, int vec) {
  using V = typename Mf<R>::V;
  constexpr int P = kPBrick / 64;
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
    for (int piece = 0; piece < P; ++piece) {
      const int64_t pb = p0 + piece * 64;
      cplx<R> y[16], f[16];
      load_piece<cplx<R>, G>(Ys + pb, 4 * G, G * q, nd - pb, vec_ok, y);
      load_piece<cplx<R>, G>(pbval + (((jo / 16 + jt) * P + piece) * (16 / G)) * (64 * G) + lane * G, 64 * G, 0, 64,
                             true, f);
      for (int kk = 0; kk < 16; ++kk) {
        c0 = Mf<R>::mfma(f[kk].re, y[kk].re, c0);
        c1 = Mf<R>::mfma(f[kk].im, y[kk].im, c1);
        c2 = Mf<R>::mfma(f[kk].re, y[kk].im, c2);
        c3 = Mf<R>::mfma(f[kk].im, y[kk].re, c3);
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
  auto run = [&](auto g) {
    constexpr int G = decltype(g)::value;
    if constexpr (sizeof(T) == sizeof(typename real_of<T>::type))
      launch_k(k_proj_brick<T, G>, (unsigned)npb * nst, 256, 0, st, Y, ld, ncol, c.d_pboff, c.d_pbnj,
               (const T*)c.d_pbval[ik], c.d_pdest, part, c.p.ns, c.nd, nst, vec);
    else
      launch_k(k_proj_brick_c<typename real_of<T>::type, G>, (unsigned)npb * nst, 256, 0, st, Y, ld, ncol,
               c.d_pboff, c.d_pbnj, (const T*)c.d_pbval[ik], c.d_pdest, part, c.p.ns, c.nd, nst, vec);
  };
  switch (c.pgroup) {
    case 2: run(std::integral_constant<int, 2>()); break;
    case 4: run(std::integral_constant<int, 4>()); break;
    default: run(std::integral_constant<int, 16>()); break;
  }
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
