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

// the 16 step operands of the state row Ys on piece sbk (a 64-point brick):
// local indices 4G i + G q .. + G-1 (consecutive in memory), zeros outside
// the grid
template <typename T, int G>
__device__ __forceinline__ void load_rows(const T* __restrict__ Ys, const BrickGeo& geo, int64_t sbk, int q,
                                          int64_t nd, bool vec, T* out) {
  if (!geo.cube) {
    const int64_t pb = sbk * 64;
    load_piece<T, G>(Ys + pb, 4 * G, G * q, nd - pb, vec, out);
    return;
  }
  if (sbk >= geo.nbrick) {
    for (int i = 0; i < 16; ++i) out[i] = T();
    return;
  }
  const int64_t base = geo.base(sbk);
  for (int i = 0; i < 16 / G; ++i) ld_group<T, G>(Ys + base + geo.off(4 * G * i + G * q), vec, out + G * i);
}

template <typename T, int G>
__global__ __launch_bounds__(256) void k_proj_brick(const T* __restrict__ Y, int64_t ld, int ncol,
                                                    const int64_t* __restrict__ pboff, const int* __restrict__ pbnj,
                                                    const T* __restrict__ pbval, const int64_t* __restrict__ pdest,
                                                    T* __restrict__ part, int ldp, int64_t nd, int nst, int vec,
                                                    const BrickGeo geo) {
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
        T bk[16];
        load_rows<T, G>(Ys, geo, (int64_t)b * P + piece, q, nd, vec_ok, bk);
        for (int t = 0; t < 4; ++t) {
          if (jg + t >= ntile) break;   // wave-uniform
          T a[16];
          load_piece<T, G>(trow(jg + t, piece), 64 * G, 0, 64, true, a);
          for (int kk = 0; kk < 16; ++kk) acc[t] = Mf<T>::mfma(a[kk], bk[kk], acc[t]);
        }
      }
      for (int t = 0; t < 4; ++t) {
        if (jg + t >= ntile) break;
        int64_t dst[4];   // destination rows first (clamped), then the stores
        for (int r = 0; r < 4; ++r) {
          const int j = (jg + t) * 16 + Mf<T>::row(lane, r);
          dst[r] = pdest[jo + (j < nj ? j : nj - 1)];
        }
        for (int r = 0; r < 4; ++r) {
          const int j = (jg + t) * 16 + Mf<T>::row(lane, r);
          if (j < nj && sb < ncol) part[dst[r] * ldp + sb] = acc[t][r];
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
        T bk[16], a0[16], a1[16];
        load_rows<T, G>(Ys, geo, (int64_t)b * P + piece, q, nd, vec_ok, bk);
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
      for (int t = 0; t < (two ? 2 : 1); ++t) {
        int64_t dst[4];   // destination rows first (clamped), then the stores
        for (int r = 0; r < 4; ++r) {
          const int j = (jg + t) * 16 + Mf<T>::row(lane, r);
          dst[r] = pdest[jo + (j < nj ? j : nj - 1)];
        }
        for (int r = 0; r < 4; ++r) {
          const int j = (jg + t) * 16 + Mf<T>::row(lane, r);
          if (j < nj && sb < ncol) part[dst[r] * ldp + sb] = acc[t][0][r] + acc[t][1][r];
        }
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
                                                      int ldp, int64_t nd, int nst, int vec,
                                                      const BrickGeo geo) {
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
  const cplx<R>* __restrict__ Ys = Y + (int64_t)min(sb, ncol - 1) * ld;
  const bool vec_ok = vec != 0;
  // one slot tile per sweep with four independent accumulators
  // (Re Phi Re y, Im Phi Im y, Re Phi Im y, Im Phi Re y)
  for (int jt = 0; jt < ntile; ++jt) {
    V c0, c1, c2, c3;
    for (int r = 0; r < 4; ++r) c0[r] = c1[r] = c2[r] = c3[r] = R(0);
    for (int piece = 0; piece < P; ++piece) {
      cplx<R> y[16], f[16];
      load_rows<cplx<R>, G>(Ys, geo, (int64_t)b * P + piece, q, nd, vec_ok, y);
      load_piece<cplx<R>, G>(pbval + (((jo / 16 + jt) * P + piece) * (16 / G)) * (64 * G) + lane * G, 64 * G, 0, 64,
                             true, f);
      for (int kk = 0; kk < 16; ++kk) {
        c0 = Mf<R>::mfma(f[kk].re, y[kk].re, c0);
        c1 = Mf<R>::mfma(f[kk].im, y[kk].im, c1);
        c2 = Mf<R>::mfma(f[kk].re, y[kk].im, c2);
        c3 = Mf<R>::mfma(f[kk].im, y[kk].re, c3);
      }
    }
    int64_t dst[4];   // destination rows first (clamped), then the stores
    for (int r = 0; r < 4; ++r) {
      const int j = jt * 16 + Mf<R>::row(lane, r);
      dst[r] = pdest[jo + (j < nj ? j : nj - 1)];
    }
    for (int r = 0; r < 4; ++r) {
      const int j = jt * 16 + Mf<R>::row(lane, r);
      if (j < nj && sb < ncol) part[dst[r] * ldp + sb] = cplx<R>(c0[r] + c1[r], c2[r] - c3[r]);
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

// ------------------------------------------------ fused scatter + projection
// Real blocks inside a Chebyshev step: the projector scatter of this step's
// output and the projections of that output (the next step's input) in one
// pass,
//   Y_b += alpha Phi_b Q                   (64-point bricks, as k_nl_brick)
//   part[pdest[slot]][s] = sum_{p in B} Phi[slot][p] Y[s][p]
//                                           (256-point brick B, as k_proj_brick)
// One workgroup per (projection brick, 64 states) walks the brick's four
// scatter bricks.  For each, the coupled projections alpha Q of the brick's
// functions (for the workgroup's 64 states) and the brick's table rows are
// staged into LDS by all four waves together, a chunk of functions at a
// time (one batched round trip to memory per chunk, each value fetched once
// per workgroup), and the waves' matrix-core updates of their 16 states read
// both operands from LDS.  The updated values are written back and, through
// a wave-private LDS tile [state][point] (rows padded by 16 bytes) that
// reuses the staging area, fed into the projection's operand order, so the
// block is read and written once for both operations.  NT bounds the
// brick's slot tiles (all projection accumulators stay in registers).
template <typename T> constexpr int kYsRow = kBrick + 16 / (int)sizeof(T);
template <typename T> constexpr int kStageFns = sizeof(T) == 8 ? 32 : 64;   // functions staged per chunk

// body of one workgroup: projection brick b, state tile st_; DB: FP32 slot
// tiles' table values double-buffered (off where the register budget has no
// room: the multi-job kernel)
template <typename T, int G, int NT, bool DB = true>
__device__ __forceinline__ void fused_real(const BrickGeo& geo, T* __restrict__ Y, int64_t ld, int ncol,
                                           const int64_t* __restrict__ boff,
                                           const int* __restrict__ bnj, const int* __restrict__ bj,
                                           const T* __restrict__ bval, const T* __restrict__ Qt, int ldq, T alpha,
                                           int nbrick, const int64_t* __restrict__ pboff,
                                           const int* __restrict__ pbnj, const T* __restrict__ pbval,
                                           const int64_t* __restrict__ pdest, T* __restrict__ part, int ldp,
                                           int64_t nd, int b, int st_) {
  using V = typename Mf<T>::V;
  constexpr int P = kPBrick / kBrick;
  constexpr int RS = kYsRow<T>;                // row of a transposition tile and of a staged function
  constexpr int CH = kStageFns<T>;
  constexpr int kYs = 4 * 16 * RS, kSt = 2 * CH * RS;
  __shared__ __attribute__((aligned(16))) T lds[kYs > kSt ? kYs : kSt];
  T* const sQ = lds;             // [CH][RS]: alpha Q of the chunk's functions, the workgroup's states
  T* const sB = lds + CH * RS;   // [CH][RS]: the chunk's rows of the brick's value table
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int swg = st_ * 64;
  const int s0 = swg + wave * 16;
  // waves past the last state take part in the staging and the barriers only
  const bool wave_ok = s0 < ncol;
  const int sa = s0 + (lane & 15);
  const bool sa_ok = sa < ncol;
  const int q = lane >> 4;
  const int njp = pbnj[b];
  const int ntile = (njp + 15) / 16;   // <= NT (host-checked)
  const int64_t jop = pboff[b];
  T* const yw = lds + wave * 16 * RS;
  V pacc[NT];
  for (int t = 0; t < NT; ++t)
    for (int r = 0; r < 4; ++r) pacc[t][r] = T(0);
  // FP64: the scatter bricks' table offsets and (padded) function counts,
  // all P of them at once (clamped to the last brick; bricks past it are
  // not used), and each brick's first-chunk function indices requested one
  // brick ahead.  FP32 loads both where they are used: with its 64-function
  // chunks the carried indices cost more scalar registers than the round
  // trips they save (c3 measured slower).
  constexpr bool kIdx = sizeof(T) == 8;
  int64_t jo_k[P];
  int nj4_k[P];
  if constexpr (kIdx)
    for (int k = 0; k < P; ++k) {
      const int sbk = min(b * P + k, nbrick - 1);
      jo_k[k] = boff[sbk];
      nj4_k[k] = (bnj[sbk] + 3) & ~3;
    }
  // Function indices of a brick's first chunk: one per lane by a vector load
  // (clamped inside the index array, which has a tail past the last brick),
  // then the wave's own as uniform values.  The next brick's are requested
  // while the current one is processed, so they arrive with the current
  // brick's staging loads and are read out after its chunk loop.
  constexpr int NJ = CH / 4;
  auto chunk0_idx = [&](int k) -> int {
    const int nc = min(CH, nj4_k[k]);
    return bj[jo_k[k] + (lane < nc ? lane : max(nc - 1, 0))];
  };
  int jgs[NJ];
  if constexpr (kIdx) {
    const int v = chunk0_idx(0);
    for (int i = 0; i < NJ; ++i) jgs[i] = __builtin_amdgcn_readlane(v, wave + 4 * i);
  }
  int bj_next = 0;
  for (int k = 0; k < P; ++k) {
    const int sbk = b * P + k;
    if (sbk >= nbrick) break;   // uniform: the last brick of a ragged grid
    const int64_t p0 = geo.base(sbk);   // local index pt*16 + lane%16 at p0 + geo.off(...)
    // ---- scatter of brick sbk
    V acc[4];
    for (int pt = 0; pt < 4; ++pt)
      for (int r = 0; r < 4; ++r) {
        const int s = s0 + Mf<T>::row(lane, r);
        const int64_t p = p0 + geo.off(pt * 16 + (lane & 15));
        acc[pt][r] = (s < ncol && p < nd) ? Y[(int64_t)s * ld + p] : T(0);
      }
    const int64_t jo = kIdx ? jo_k[k] : boff[sbk];
    const int nj4 = kIdx ? nj4_k[k] : (bnj[sbk] + 3) & ~3;   // uniform over the workgroup
    const T* __restrict__ vb = bval + jo * kBrick;
    if (kIdx && k + 1 < P) bj_next = chunk0_idx(k + 1);
    for (int c0 = 0; c0 < nj4; c0 += CH) {
      const int nc = min(CH, nj4 - c0);
      // Every load of the chunk is issued before the first LDS write, from
      // clamped in-range addresses, and out-of-range entries are zeroed by
      // selection: conditional loads become branches, each closed by a wait
      // for all outstanding loads, which serialises the chunk's round trips.
      constexpr int NB = (sizeof(T) == 8 && NT > 4) ? 2 : 1;   // load batches (register budget)
      constexpr int NI = CH / 4 / NB;
      const int s = swg + lane;
      const int sc = s < ncol ? s : ncol - 1;
      __syncthreads();   // earlier readers of the area (staging or transposition tiles) are done
      for (int h = 0; h < NB; ++h) {
        int jg[NI];
        if (kIdx && c0 == 0) {
          for (int i = 0; i < NI; ++i) jg[i] = jgs[h * NI + i];
        } else {
          for (int i = 0; i < NI; ++i) {
            const int fn = wave + 4 * (h * NI + i);   // wave-uniform
            jg[i] = bj[jo + c0 + (fn < nc ? fn : nc - 1)];
          }
        }
        __builtin_amdgcn_sched_barrier(0);   // the index loads go out together
        T qraw[NI], braw[NI];
        for (int i = 0; i < NI; ++i) {
          const int fn = wave + 4 * (h * NI + i);
          qraw[i] = Qt[(int64_t)(jg[i] >= 0 ? jg[i] : 0) * ldq + sc];
          braw[i] = vb[(int64_t)(c0 + (fn < nc ? fn : nc - 1)) * kBrick + lane];
        }
        __builtin_amdgcn_sched_barrier(0);   // and the value loads before any use
        for (int i = 0; i < NI; ++i) {
          const int fn = wave + 4 * (h * NI + i);
          sQ[fn * RS + lane] = (fn < nc && jg[i] >= 0 && s < ncol) ? alpha * qraw[i] : T(0);
          sB[fn * RS + lane] = fn < nc ? braw[i] : T(0);
        }
      }
      __syncthreads();
      if (wave_ok)
        for (int f4 = 0; f4 < nc; f4 += 4) {
          const int fr = (f4 + q) * RS;
          const T a = sQ[fr + wave * 16 + (lane & 15)];
          for (int pt = 0; pt < 4; ++pt) acc[pt] = Mf<T>::mfma(a, sB[fr + pt * 16 + (lane & 15)], acc[pt]);
        }
    }
    if (kIdx && k + 1 < P)   // the next brick's chunk-0 indices (their load has completed)
      for (int i = 0; i < NJ; ++i) jgs[i] = __builtin_amdgcn_readlane(bj_next, wave + 4 * i);
    __syncthreads();   // the staging area becomes the transposition tiles
    for (int pt = 0; pt < 4; ++pt)
      for (int r = 0; r < 4; ++r) {
        const int sl = Mf<T>::row(lane, r);
        const int64_t p = p0 + geo.off(pt * 16 + (lane & 15));
        if (nj4 > 0 && s0 + sl < ncol && p < nd) Y[(int64_t)(s0 + sl) * ld + p] = acc[pt][r];
        yw[sl * RS + pt * 16 + (lane & 15)] = acc[pt][r];
      }
    if (ntile == 0 || !wave_ok) continue;
    // ---- projection of the updated piece k (wave-private LDS, in order)
    wave_lds_sync();   // every lane's writes of yw are visible
    T bk[16];
    load_piece<T, G>(yw + (lane & 15) * RS, 4 * G, G * q, 64, true, bk);
    auto tab = [&](int t) { return pbval + (((jop / 16 + t) * P + k) * (16 / G)) * (64 * G) + lane * G; };
    if constexpr (sizeof(T) == 4 && DB) {
      // FP32: slot tile t+1's table values are requested before tile t's
      // products (16 more registers, still three waves per SIMD), so the
      // tiles' round trips to the table overlap instead of adding up
      T a[2][16];
      load_piece<T, G>(tab(0), 64 * G, 0, 64, true, a[0]);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (t >= ntile) break;   // wave-uniform
        if (t + 1 < ntile) load_piece<T, G>(tab(t + 1), 64 * G, 0, 64, true, a[(t + 1) & 1]);
        for (int kk = 0; kk < 16; ++kk) pacc[t] = Mf<T>::mfma(a[t & 1][kk], bk[kk], pacc[t]);
      }
    } else if constexpr (DB && NT <= 4) {
      // FP64: only the first half of each slot tile (steps 0-7) is
      // double-buffered (16 registers, three waves per SIMD kept): tile t+1's
      // first half is requested before tile t's products and each tile's
      // second half at its start, covered by the products of the first half
      constexpr int HG = 8 / G;   // load groups per half
      auto half = [&](int t, int h, T* out) {
        for (int i = 0; i < HG; ++i) ld_group<T, G>(tab(t) + (h * HG + i) * (64 * G), true, out + G * i);
      };
      T alo[2][8], ahi[8];
      half(0, 0, alo[0]);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (t >= ntile) break;   // wave-uniform
        half(t, 1, ahi);
        if (t + 1 < ntile) half(t + 1, 0, alo[(t + 1) & 1]);
        for (int kk = 0; kk < 8; ++kk) pacc[t] = Mf<T>::mfma(alo[t & 1][kk], bk[kk], pacc[t]);
        for (int kk = 0; kk < 8; ++kk) pacc[t] = Mf<T>::mfma(ahi[kk], bk[8 + kk], pacc[t]);
      }
    } else {
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (t >= ntile) break;   // wave-uniform
        T a[16];
        load_piece<T, G>(tab(t), 64 * G, 0, 64, true, a);
        for (int kk = 0; kk < 16; ++kk) pacc[t] = Mf<T>::mfma(a[kk], bk[kk], pacc[t]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (t >= ntile) break;
    int64_t dst[4];   // destination rows first (clamped), then the stores
    for (int r = 0; r < 4; ++r) {
      const int j = t * 16 + Mf<T>::row(lane, r);
      dst[r] = pdest[jop + (j < njp ? j : njp - 1)];
    }
    for (int r = 0; r < 4; ++r) {
      const int j = t * 16 + Mf<T>::row(lane, r);
      if (j < njp && sa_ok) part[dst[r] * ldp + sa] = pacc[t][r];
    }
  }
}

template <typename T, int G, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_scatter_project(
    T* __restrict__ Y, int64_t ld, int ncol, const int64_t* __restrict__ boff, const int* __restrict__ bnj,
    const int* __restrict__ bj, const T* __restrict__ bval, const T* __restrict__ Qt, int ldq, T alpha, int nbrick,
    const int64_t* __restrict__ pboff, const int* __restrict__ pbnj, const T* __restrict__ pbval,
    const int64_t* __restrict__ pdest, T* __restrict__ part, int ldp, int64_t nd, int nst, const BrickGeo geo) {
  const unsigned lw = xcd_linear();   // 1-D grid: state tile fastest, then brick
  fused_real<T, G, NT>(geo, Y, ld, ncol, boff, bnj, bj, bval, Qt, ldq, alpha, nbrick, pboff, pbnj, pbval, pdest, part,
                       ldp, nd, lw / nst, lw % nst);
}

// The job whose workgroups contain lw (jobs ordered by first workgroup).
__device__ __forceinline__ const FusedJob& fused_job(const FusedJob* __restrict__ jobs, int njob, unsigned lw) {
  int lo = 0, hi = njob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].item0 <= lw) lo = mid;
    else hi = mid - 1;
  }
  return jobs[lo];
}

// One launch over the blocks of several (cell, spin, k) problems: the
// workgroups of job i are item0_i .. item0_{i+1} - 1 (XCD-contiguous).
template <typename T, int G, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_scatter_project_batch(
    const FusedJob* __restrict__ jobs, int njob) {
  const unsigned lw = xcd_linear();
  const FusedJob& J = fused_job(jobs, njob, lw);
  const unsigned local = lw - J.item0;
  fused_real<T, G, NT, false>(J.geo, (T*)J.Y, J.ld, J.ncol, J.boff, J.bnj, J.bj, (const T*)J.bval, (const T*)J.Qt, J.ldq,
                       (T)J.alpha, J.nbrick, J.pboff, J.pbnj, (const T*)J.pbval, J.pdest, (T*)J.part, J.ldp, J.nd,
                       local / J.nst, local % J.nst);
}

// Complex (Bloch) blocks in FP32: the same fused pass with the scatter's
// four real products per step (k_nl_brick_c) and the projection's four
// accumulators per slot tile (k_proj_brick_c); at most four slot tiles.  The
// scatter's operands are staged into LDS by the four waves together, a chunk
// of functions at a time, as for real blocks (two batches of loads per
// chunk: the projection accumulators leave less register room).  Both
// complex products take three real ones (Gauss): u v with
//   Re = Σ ur vr − Σ ui vi,  Im = Σ (ur + ui)(vr + vi) − Σ ur vr − Σ ui vi,
// a quarter fewer matrix-core products and accumulators.
template <typename R, int G, int NT>
__device__ __forceinline__ void fused_cplx(const BrickGeo& geo, cplx<R>* __restrict__ Y, int64_t ld, int ncol,
                                           const int64_t* __restrict__ boff, const int* __restrict__ bnj,
                                           const int* __restrict__ bj, const cplx<R>* __restrict__ bval,
                                           const cplx<R>* __restrict__ Qt, int ldq, R alpha, int nbrick,
                                           const int64_t* __restrict__ pboff, const int* __restrict__ pbnj,
                                           const cplx<R>* __restrict__ pbval, const int64_t* __restrict__ pdest,
                                           cplx<R>* __restrict__ part, int ldp, int64_t nd, int b, int st_) {
  using V = typename Mf<R>::V;
  using C = cplx<R>;
  constexpr int P = kPBrick / kBrick;
  constexpr int RS = kYsRow<C>;
  constexpr int CH = kStageFns<C>;
  constexpr int kYs = 4 * 16 * RS, kSt = 2 * CH * RS;
  __shared__ __attribute__((aligned(16))) unsigned char lds_raw[(kYs > kSt ? kYs : kSt) * sizeof(C)];
  C* const lds = reinterpret_cast<C*>(lds_raw);
  C* const sQ = lds;             // [CH][RS]: alpha Q of the chunk's functions, the workgroup's states
  C* const sB = lds + CH * RS;   // [CH][RS]: the chunk's rows of the brick's value table
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int swg = st_ * 64;
  const int s0 = swg + wave * 16;
  // waves past the last state take part in the staging and the barriers only
  const bool wave_ok = s0 < ncol;
  const int sa = s0 + (lane & 15);
  const bool sa_ok = sa < ncol;
  const int q = lane >> 4;
  const int njp = pbnj[b];
  const int ntile = (njp + 15) / 16;   // <= NT (host-checked)
  const int64_t jop = pboff[b];
  C* const yw = lds + wave * 16 * RS;
  // per slot tile: sums of Re Phi Re y, Im Phi Im y, (Re Phi - Im Phi)(Re y + Im y)
  V pc[NT][3];
  for (int t = 0; t < NT; ++t)
    for (int h = 0; h < 3; ++h)
      for (int r = 0; r < 4; ++r) pc[t][h][r] = R(0);
  for (int k = 0; k < P; ++k) {
    const int sbk = b * P + k;
    if (sbk >= nbrick) break;   // uniform: the last brick of a ragged grid
    const int64_t p0 = geo.base(sbk);   // local index pt*16 + lane%16 at p0 + geo.off(...)
    // ---- scatter of brick sbk (k_nl_brick_c's steps)
    // Loads from clamped in-range addresses, zeroed by selection afterwards
    // (a conditional load becomes a branch closed by a wait for every
    // outstanding load, one round trip per value).
    // Y + alpha Phi Q as three sums started from Y: s1 = Re Y + Σ Re q Re f,
    // s2 = Σ Im q Im f, s3 = Re Y + Im Y + Σ (Re q + Im q)(Re f + Im f);
    // the result is (s1 - s2, s3 - s1 - s2)
    V s1[4], s2[4], s3[4];
    {
      C yv[4][4];
      for (int pt = 0; pt < 4; ++pt)
        for (int r = 0; r < 4; ++r) {
          const int s = min(s0 + Mf<R>::row(lane, r), ncol - 1);
          const int64_t p = min(p0 + geo.off(pt * 16 + (lane & 15)), nd - 1);
          yv[pt][r] = Y[(int64_t)s * ld + p];
        }
      for (int pt = 0; pt < 4; ++pt)
        for (int r = 0; r < 4; ++r) {
          const bool in = s0 + Mf<R>::row(lane, r) < ncol && p0 + geo.off(pt * 16 + (lane & 15)) < nd;
          const R yr = in ? yv[pt][r].re : R(0), yi = in ? yv[pt][r].im : R(0);
          s1[pt][r] = yr;
          s2[pt][r] = R(0);
          s3[pt][r] = yr + yi;
        }
    }
    const int64_t jo = boff[sbk];
    const int nj4 = (bnj[sbk] + 3) & ~3;   // uniform over the workgroup
    const C* __restrict__ vb = bval + jo * kBrick;
    for (int c0 = 0; c0 < nj4; c0 += CH) {
      const int nc = min(CH, nj4 - c0);
      // the chunk's loads from clamped in-range addresses, all issued before
      // the first LDS write; out-of-range entries zeroed by selection
      constexpr int NB = 2, NI = CH / 4 / NB;
      const int s = swg + lane;
      const int sc = s < ncol ? s : ncol - 1;
      __syncthreads();   // earlier readers of the area (staging or transposition tiles) are done
      for (int h = 0; h < NB; ++h) {
        int jg[NI];
        for (int i = 0; i < NI; ++i) {
          const int fn = wave + 4 * (h * NI + i);   // wave-uniform
          jg[i] = bj[jo + c0 + (fn < nc ? fn : nc - 1)];
        }
        __builtin_amdgcn_sched_barrier(0);   // the index loads go out together
        C qraw[NI], braw[NI];
        for (int i = 0; i < NI; ++i) {
          const int fn = wave + 4 * (h * NI + i);
          qraw[i] = Qt[(int64_t)(jg[i] >= 0 ? jg[i] : 0) * ldq + sc];
          braw[i] = vb[(int64_t)(c0 + (fn < nc ? fn : nc - 1)) * kBrick + lane];
        }
        __builtin_amdgcn_sched_barrier(0);   // and the value loads before any use
        for (int i = 0; i < NI; ++i) {
          const int fn = wave + 4 * (h * NI + i);
          const bool qok = fn < nc && jg[i] >= 0 && s < ncol;
          sQ[fn * RS + lane] = qok ? C(alpha * qraw[i].re, alpha * qraw[i].im) : C(R(0), R(0));
          sB[fn * RS + lane] = fn < nc ? braw[i] : C(R(0), R(0));
        }
      }
      __syncthreads();
      if (wave_ok)
        for (int f4 = 0; f4 < nc; f4 += 4) {
          const int fr = (f4 + q) * RS;
          const C a = sQ[fr + wave * 16 + (lane & 15)];
          const R asum = a.re + a.im;
          C f[4];
          for (int pt = 0; pt < 4; ++pt) f[pt] = sB[fr + pt * 16 + (lane & 15)];
          for (int pt = 0; pt < 4; ++pt) {
            s1[pt] = Mf<R>::mfma(a.re, f[pt].re, s1[pt]);
            s2[pt] = Mf<R>::mfma(a.im, f[pt].im, s2[pt]);
            s3[pt] = Mf<R>::mfma(asum, f[pt].re + f[pt].im, s3[pt]);
          }
        }
    }
    __syncthreads();   // the staging area becomes the transposition tiles
    for (int pt = 0; pt < 4; ++pt)
      for (int r = 0; r < 4; ++r) {
        const int sl = Mf<R>::row(lane, r);
        const int64_t p = p0 + geo.off(pt * 16 + (lane & 15));
        const C v(s1[pt][r] - s2[pt][r], s3[pt][r] - s1[pt][r] - s2[pt][r]);
        if (nj4 > 0 && s0 + sl < ncol && p < nd) Y[(int64_t)(s0 + sl) * ld + p] = v;
        yw[sl * RS + pt * 16 + (lane & 15)] = v;
      }
    if (ntile == 0 || !wave_ok) continue;
    // ---- projection of the updated piece k (wave-private LDS, in order)
    wave_lds_sync();   // every lane's writes of yw are visible
    C y[16];
    load_piece<C, G>(yw + (lane & 15) * RS, 4 * G, G * q, 64, true, y);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (t >= ntile) break;   // wave-uniform
      C f[16];
      load_piece<C, G>(pbval + (((jop / 16 + t) * P + k) * (16 / G)) * (64 * G) + lane * G, 64 * G, 0, 64, true,
                       f);
      for (int kk = 0; kk < 16; ++kk) {
        pc[t][0] = Mf<R>::mfma(f[kk].re, y[kk].re, pc[t][0]);
        pc[t][1] = Mf<R>::mfma(f[kk].im, y[kk].im, pc[t][1]);
        pc[t][2] = Mf<R>::mfma(f[kk].re - f[kk].im, y[kk].re + y[kk].im, pc[t][2]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (t >= ntile) break;
    int64_t dst[4];   // destination rows first (clamped), then the stores
    for (int r = 0; r < 4; ++r) {
      const int j = t * 16 + Mf<R>::row(lane, r);
      dst[r] = pdest[jop + (j < njp ? j : njp - 1)];
    }
    for (int r = 0; r < 4; ++r) {
      const int j = t * 16 + Mf<R>::row(lane, r);
      // conj(Phi) y = (Σ Re Re + Σ Im Im, Σ (Re - Im)(Re + Im) - Σ Re Re + Σ Im Im)
      if (j < njp && sa_ok)
        part[dst[r] * ldp + sa] = C(pc[t][0][r] + pc[t][1][r], pc[t][2][r] - pc[t][0][r] + pc[t][1][r]);
    }
  }
}

template <typename R, int G, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_scatter_project_c(
    cplx<R>* __restrict__ Y, int64_t ld, int ncol, const int64_t* __restrict__ boff, const int* __restrict__ bnj,
    const int* __restrict__ bj, const cplx<R>* __restrict__ bval, const cplx<R>* __restrict__ Qt, int ldq, R alpha,
    int nbrick, const int64_t* __restrict__ pboff, const int* __restrict__ pbnj, const cplx<R>* __restrict__ pbval,
    const int64_t* __restrict__ pdest, cplx<R>* __restrict__ part, int ldp, int64_t nd, int nst,
    const BrickGeo geo) {
  const unsigned lw = xcd_linear();
  fused_cplx<R, G, NT>(geo, Y, ld, ncol, boff, bnj, bj, bval, Qt, ldq, alpha, nbrick, pboff, pbnj, pbval, pdest, part,
                       ldp, nd, lw / nst, lw % nst);
}

template <typename R, int G, int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_scatter_project_c_batch(
    const FusedJob* __restrict__ jobs, int njob) {
  using C = cplx<R>;
  const unsigned lw = xcd_linear();
  const FusedJob& J = fused_job(jobs, njob, lw);
  const unsigned local = lw - J.item0;
  fused_cplx<R, G, NT>(J.geo, (C*)J.Y, J.ld, J.ncol, J.boff, J.bnj, J.bj, (const C*)J.bval, (const C*)J.Qt, J.ldq,
                       (R)J.alpha, J.nbrick, J.pboff, J.pbnj, (const C*)J.pbval, J.pdest, (C*)J.part, J.ldp, J.nd,
                       local / J.nst, local % J.nst);
}

template <typename T>
bool scatter_project_ok(const Ctx& c) {
  if (c.nproj == 0 || c.pboff.empty()) return false;
  if constexpr (sizeof(T) == sizeof(typename real_of<T>::type)) return c.max_ptiles <= 8;
  else if constexpr (std::is_same<T, cplx<float>>::value) return c.max_ptiles <= 4 && c.pgroup == 2;
  else return false;   // complex FP64: the accumulators do not fit the register budget
}

// part: 1 = the fused kernel only, 2 = the partial sums and coupling that
// follow it only, 3 = both (separate parts let the caller time the kernel)
template <typename T>
void launch_scatter_project(const Ctx& c, int ik, T* Y, int64_t ld, int ncol, const T* Qt, double alpha,
                            const double* coup, T* P, T* Q, hipStream_t st, int part_sel) {
  if constexpr (sizeof(T) == sizeof(typename real_of<T>::type)) {
    T* part = reinterpret_cast<T*>(c.d_ppart);
    const int npb = (int)c.pboff.size() - 1;
    const int nbrick = (int)c.boff.size() - 1;
    const int nst = (ncol + 63) / 64;
    auto run = [&](auto g, auto nt) {
      constexpr int G = decltype(g)::value, NT = decltype(nt)::value;
      launch_k(k_scatter_project<T, G, NT>, (unsigned)npb * nst, 256, 0, st, Y, ld, ncol, c.d_boff, c.d_bnj, c.d_bj,
               (const T*)c.d_bval[ik], Qt, c.p.ns, (T)alpha, nbrick, c.d_pboff, c.d_pbnj, (const T*)c.d_pbval[ik],
               c.d_pdest, part, c.p.ns, c.nd, nst, c.geo);
    };
    using I2 = std::integral_constant<int, 2>;
    using I4 = std::integral_constant<int, 4>;
    using I8 = std::integral_constant<int, 8>;
    if (part_sel & 1) {
      if (c.pgroup == 2) {
        if (c.max_ptiles <= 4) run(I2(), I4()); else run(I2(), I8());
      } else {
        if (c.max_ptiles <= 4) run(I4(), I4()); else run(I4(), I8());
      }
    }
    if (part_sel & 2) {
      dim3 g2((ncol + 63) / 64, c.nproj);
      launch_k(k_slot_sum<T>, g2, 1024, 0, st, part, c.p.ns, ncol, c.d_jrow, P, c.nproj, c.dv);
      dim3 g3((ncol + 63) / 64, (unsigned)c.blocks.size());
      launch_k(k_couple<T>, g3, 64, 0, st, P, c.d_blocks, ncol, coup, Q, c.nproj, c.p.ns);
    }
  } else if constexpr (std::is_same<T, cplx<float>>::value) {
    T* part = reinterpret_cast<T*>(c.d_ppart);
    const int npb = (int)c.pboff.size() - 1;
    const int nbrick = (int)c.boff.size() - 1;
    const int nst = (ncol + 63) / 64;
    if (part_sel & 1)
      launch_k(k_scatter_project_c<float, 2, 4>, (unsigned)npb * nst, 256, 0, st, Y, ld, ncol, c.d_boff, c.d_bnj,
               c.d_bj, (const T*)c.d_bval[ik], Qt, c.p.ns, (float)alpha, nbrick, c.d_pboff, c.d_pbnj,
               (const T*)c.d_pbval[ik], c.d_pdest, part, c.p.ns, c.nd, nst, c.geo);
    if (part_sel & 2) {
      dim3 g2((ncol + 63) / 64, c.nproj);
      launch_k(k_slot_sum<T>, g2, 1024, 0, st, part, c.p.ns, ncol, c.d_jrow, P, c.nproj, c.dv);
      dim3 g3((ncol + 63) / 64, (unsigned)c.blocks.size());
      launch_k(k_couple<T>, g3, 64, 0, st, P, c.d_blocks, ncol, coup, Q, c.nproj, c.p.ns);
    }
  }
}

template bool scatter_project_ok<double>(const Ctx&);
template bool scatter_project_ok<float>(const Ctx&);
template bool scatter_project_ok<cplx<double>>(const Ctx&);
template bool scatter_project_ok<cplx<float>>(const Ctx&);
template void launch_scatter_project<double>(const Ctx&, int, double*, int64_t, int, const double*, double,
                                             const double*, double*, double*, hipStream_t, int);
template void launch_scatter_project<float>(const Ctx&, int, float*, int64_t, int, const float*, double,
                                            const double*, float*, float*, hipStream_t, int);
template void launch_scatter_project<cplx<double>>(const Ctx&, int, cplx<double>*, int64_t, int,
                                                   const cplx<double>*, double, const double*, cplx<double>*,
                                                   cplx<double>*, hipStream_t, int);
template void launch_scatter_project<cplx<float>>(const Ctx&, int, cplx<float>*, int64_t, int, const cplx<float>*,
                                                  double, const double*, cplx<float>*, cplx<float>*, hipStream_t,
                                                  int);

// The job record of the fused pass of one block (the block's data, the
// projection partials of that block, its first workgroup).
template <typename T>
FusedJob fused_job_of(const Ctx& c, int ik, T* Y, int64_t ld, int ncol, const T* Qt, double alpha, void* part,
                      unsigned item0) {
  FusedJob j{};
  j.geo = c.geo;
  j.Y = Y; j.ld = ld; j.ncol = ncol; j.nst = (ncol + 63) / 64;
  j.boff = c.d_boff; j.bnj = c.d_bnj; j.bj = c.d_bj; j.bval = c.d_bval[ik];
  j.Qt = Qt; j.ldq = c.p.ns; j.alpha = alpha; j.nbrick = (int)c.boff.size() - 1;
  j.pboff = c.d_pboff; j.pbnj = c.d_pbnj; j.pbval = c.d_pbval[ik]; j.pdest = c.d_pdest;
  j.part = part; j.ldp = c.p.ns; j.nd = c.nd;
  j.item0 = item0;
  return j;
}

unsigned fused_job_items(const Ctx& c, int ncol) {
  return (unsigned)((c.pboff.size() - 1) * (size_t)((ncol + 63) / 64));
}

template <typename T>
void launch_scatter_project_batch(const FusedJob* d_jobs, int njob, unsigned items, int G, int NT, hipStream_t st) {
  if constexpr (sizeof(T) == sizeof(typename real_of<T>::type)) {
    if (G == 2) {
      if (NT <= 4) launch_k(k_scatter_project_batch<T, 2, 4>, items, 256, 0, st, d_jobs, njob);
      else launch_k(k_scatter_project_batch<T, 2, 8>, items, 256, 0, st, d_jobs, njob);
    } else {
      if (NT <= 4) launch_k(k_scatter_project_batch<T, 4, 4>, items, 256, 0, st, d_jobs, njob);
      else launch_k(k_scatter_project_batch<T, 4, 8>, items, 256, 0, st, d_jobs, njob);
    }
  } else if constexpr (std::is_same<T, cplx<float>>::value) {
    launch_k(k_scatter_project_c_batch<float, 2, 4>, items, 256, 0, st, d_jobs, njob);
  }
}

#define INST_FUSED_JOB(T)                                                                                    \
  template FusedJob fused_job_of<T>(const Ctx&, int, T*, int64_t, int, const T*, double, void*, unsigned);  \
  template void launch_scatter_project_batch<T>(const FusedJob*, int, unsigned, int, int, hipStream_t);
INST_FUSED_JOB(double)
INST_FUSED_JOB(float)
INST_FUSED_JOB(cplx<double>)
INST_FUSED_JOB(cplx<float>)

size_t project_partial_elems(const Ctx& c) {
  if (c.pboff.empty()) return 0;
  return (size_t)c.pboff.back() * c.p.ns;
}

// P = Phi^H Y dV with the function values of `table` (projection-brick
// layout: the context's orbitals/projectors at a k-point, or other functions
// on the same supports, e.g. their moments).
template <typename T>
void launch_project_table(const Ctx& c, const T* table, const T* Y, int ncol, int64_t ld, T* P, hipStream_t st) {
  if (c.nproj == 0) return;
  T* part = reinterpret_cast<T*>(c.d_ppart);
  const int npb = (int)c.pboff.size() - 1;
  const int nst = (ncol + 63) / 64;
  // wide loads of the state rows need 16-byte aligned rows
  const int vec = ((uintptr_t)Y % 16 == 0 && (ld * (int64_t)sizeof(T)) % 16 == 0) ? 1 : 0;
  auto run = [&](auto g) {
    constexpr int G = decltype(g)::value;
    if constexpr (sizeof(T) == sizeof(typename real_of<T>::type))
      launch_k(k_proj_brick<T, G>, (unsigned)npb * nst, 256, 0, st, Y, ld, ncol, c.d_pboff, c.d_pbnj, table,
               c.d_pdest, part, c.p.ns, c.nd, nst, vec, c.geo);
    else
      launch_k(k_proj_brick_c<typename real_of<T>::type, G>, (unsigned)npb * nst, 256, 0, st, Y, ld, ncol,
               c.d_pboff, c.d_pbnj, table, c.d_pdest, part, c.p.ns, c.nd, nst, vec, c.geo);
  };
  if (c.pgroup == 4) run(std::integral_constant<int, 4>());
  else run(std::integral_constant<int, 2>());
  dim3 g2((ncol + 63) / 64, c.nproj);
  launch_k(k_slot_sum<T>, g2, 1024, 0, st, part, c.p.ns, ncol, c.d_jrow, P, c.nproj, c.dv);
}

template <typename T>
void launch_project_brick(const Ctx& c, int ik, const T* Y, int ncol, int64_t ld, const double* coup, T* P, T* Q,
                          hipStream_t st) {
  if (c.nproj == 0) return;
  launch_project_table<T>(c, (const T*)c.d_pbval[ik], Y, ncol, ld, P, st);
  dim3 g3((ncol + 63) / 64, (unsigned)c.blocks.size());
  launch_k(k_couple<T>, g3, 64, 0, st, P, c.d_blocks, ncol, coup, Q, c.nproj, c.p.ns);
}

template <typename T>
void launch_couple(const Ctx& c, const T* P, int ncol, const double* coup, T* Q, hipStream_t st) {
  if (c.nproj == 0) return;
  dim3 g3((ncol + 63) / 64, (unsigned)c.blocks.size());
  launch_k(k_couple<T>, g3, 64, 0, st, P, c.d_blocks, ncol, coup, Q, c.nproj, c.p.ns);
}
template void launch_couple<double>(const Ctx&, const double*, int, const double*, double*, hipStream_t);
template void launch_couple<float>(const Ctx&, const float*, int, const double*, float*, hipStream_t);
template void launch_couple<cplx<double>>(const Ctx&, const cplx<double>*, int, const double*, cplx<double>*,
                                          hipStream_t);
template void launch_couple<cplx<float>>(const Ctx&, const cplx<float>*, int, const double*, cplx<float>*,
                                         hipStream_t);

template void launch_project_table<double>(const Ctx&, const double*, const double*, int, int64_t, double*,
                                           hipStream_t);
template void launch_project_table<float>(const Ctx&, const float*, const float*, int, int64_t, float*, hipStream_t);
template void launch_project_table<cplx<double>>(const Ctx&, const cplx<double>*, const cplx<double>*, int, int64_t,
                                                 cplx<double>*, hipStream_t);
template void launch_project_table<cplx<float>>(const Ctx&, const cplx<float>*, const cplx<float>*, int, int64_t,
                                                cplx<float>*, hipStream_t);

template void launch_project_brick<double>(const Ctx&, int, const double*, int, int64_t, const double*, double*,
                                           double*, hipStream_t);
template void launch_project_brick<float>(const Ctx&, int, const float*, int, int64_t, const double*, float*,
                                          float*, hipStream_t);
template void launch_project_brick<cplx<double>>(const Ctx&, int, const cplx<double>*, int, int64_t, const double*,
                                                 cplx<double>*, cplx<double>*, hipStream_t);
template void launch_project_brick<cplx<float>>(const Ctx&, int, const cplx<float>*, int, int64_t, const double*,
                                                cplx<float>*, cplx<float>*, hipStream_t);

}  // namespace hcu
