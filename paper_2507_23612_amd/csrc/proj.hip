// Projections of a block of states onto the atom-centred functions, one atom
// block at a time (Sec. II.B: all integrals of one atom are computed together,
// atom after atom, as for nonlocal projectors):
//
//   P[s][j0+m] = dV * sum_{q in supp} conj(phi_m(x_q)) y_s(x_q)          (trapezoid rule)
//   Q[j0+m][s] = sum_m' C_b[m][m'] P[s][j0+m']     (Q stored transposed for the scatter)
//
// with C_b = diag(gamma) for the KB channels and C_b = U (1/2 - D) for the
// Hubbard manifold (Eq. DerED).  A workgroup owns one block, S states and one
// 4096-point chunk of the block's sorted support (x-runs are contiguous): it
// holds the NM x S partial sums per thread, reduces them across the
// workgroup and writes them per chunk; a second kernel sums the chunks in a
// fixed order (deterministic) and applies the coupling.
#include "common.h"

#include <algorithm>

namespace hcu {

template <typename T>
__device__ inline T shfl_xor_t(T v, int m) { return __shfl_xor(v, m, 64); }
template <typename R>
__device__ inline cplx<R> shfl_xor_t(cplx<R> v, int m) {
  return cplx<R>(__shfl_xor(v.re, m, 64), __shfl_xor(v.im, m, 64));
}

constexpr int kChunk = 4096;   // support points per workgroup

// Stage 1: partial sums over one chunk of one block's support for S states,
// written (unscaled) to part[chunk][j][s].
template <typename T, int NM, int S>
__global__ __launch_bounds__(256) void k_project(const T* __restrict__ Y, int64_t ld, int ncol,
                                                 const BlockDesc* __restrict__ blocks,
                                                 const int* __restrict__ blist, const int* __restrict__ supp,
                                                 const T* __restrict__ cscv, T* __restrict__ part, int nproj,
                                                 int ldp) {
  // logical order: state tile fastest, then block, then chunk; XCD-contiguous
  // so the state tiles reading one support chunk share its values in one L2
  const unsigned lw = xcd_linear();
  const int stile = lw % gridDim.y;
  const int bi = (lw / gridDim.y) % gridDim.x;
  const int chunk = lw / (gridDim.x * gridDim.y);
  const BlockDesc& b = blocks[blist[bi]];
  const int s0 = stile * S;
  const int q0 = chunk * kChunk;
  if (q0 >= b.nsupp) return;
  const int q1 = min(b.nsupp, q0 + kChunk);
  const int ns_here = min(S, ncol - s0);
  T acc[NM][S];
  for (int m = 0; m < NM; ++m)
    for (int s = 0; s < S; ++s) acc[m][s] = T(0);
  const int nsupp = b.nsupp;
  const int* __restrict__ sp = supp + b.supp_off;
  const T* __restrict__ v = cscv + b.val_off;
  const T* __restrict__ Ys = Y + (int64_t)s0 * ld;
  for (int q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
    const int idx = sp[q];
    T phi[NM];
    for (int m = 0; m < NM; ++m) phi[m] = conj_(v[(int64_t)m * nsupp + q]);
    if (ns_here == S) {
      for (int s = 0; s < S; ++s) {
        const T x = Ys[(int64_t)s * ld + idx];
        for (int m = 0; m < NM; ++m) acc[m][s] += phi[m] * x;
      }
    } else {
      for (int s = 0; s < S; ++s) {
        if (s < ns_here) {
          const T x = Ys[(int64_t)s * ld + idx];
          for (int m = 0; m < NM; ++m) acc[m][s] += phi[m] * x;
        }
      }
    }
  }
  // wave reduction, then across the (up to 4) waves of the workgroup
  // raw LDS storage (T may have a constructor)
  __shared__ __attribute__((aligned(16))) unsigned char red_raw[4 * NM * S * sizeof(T)];
  T(*red)[NM * S] = reinterpret_cast<T(*)[NM * S]>(red_raw);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int m = 0; m < NM; ++m)
    for (int s = 0; s < S; ++s) {
      T x = acc[m][s];
      for (int off = 32; off > 0; off >>= 1) x += shfl_xor_t(x, off);
      if (lane == 0) red[wave][m * S + s] = x;
    }
  __syncthreads();
  const int nw = (blockDim.x + 63) / 64;
  T* __restrict__ out = part + (int64_t)chunk * nproj * ldp;
  for (int t = threadIdx.x; t < NM * S; t += blockDim.x) {
    const int m = t / S, s = t % S;
    if (s >= ns_here) continue;
    T x = red[0][t];
    for (int w = 1; w < nw; ++w) x += red[w][t];
    out[(int64_t)(b.j0 + m) * ldp + s0 + s] = x;
  }
}

// Stage 2: P[s][j] = dV * sum over the block's chunks (fixed order);
// Q[j][s] = sum_m' C_b[m][m'] P[s][j0+m'].  One thread per (block, state).
template <typename T>
__global__ void k_project_finish(const T* __restrict__ part, const BlockDesc* __restrict__ blocks, int ncol,
                                 const double* __restrict__ coup, T* __restrict__ P, T* __restrict__ Q, int nproj,
                                 int ldp, double dv) {
  const BlockDesc& b = blocks[blockIdx.y];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ncol) return;
  const int nch = (b.nsupp + kChunk - 1) / kChunk;
  using R = typename real_of<T>::type;
  T pv[kMaxNm];
  for (int m = 0; m < b.nm; ++m) {
    T x = T(0);
    for (int ch = 0; ch < nch; ++ch) x += part[(int64_t)ch * nproj * ldp + (int64_t)(b.j0 + m) * ldp + s];
    pv[m] = (R)dv * x;
    P[(int64_t)s * nproj + b.j0 + m] = pv[m];
  }
  const double* cb = coup + b.coup_off;
  for (int m = 0; m < b.nm; ++m) {
    T qv = T(0);
    for (int mp = 0; mp < b.nm; ++mp) qv += (R)cb[m * b.nm + mp] * pv[mp];
    Q[(int64_t)(b.j0 + m) * ldp + s] = qv;
  }
}

template <typename T, int NM>
static void launch_nm(const Ctx& c, const T* Y, int ncol, int64_t ld, const T* cscv, T* part, const int* d_list,
                      int nblk, int maxch, hipStream_t st) {
  constexpr int S = (sizeof(T) > 8 || NM > 5) ? 4 : 8;
  dim3 grid(nblk, (ncol + S - 1) / S, maxch);
  k_project<T, NM, S><<<grid, 256, 0, st>>>(Y, ld, ncol, c.d_blocks, d_list, c.d_supp, cscv, part, c.nproj, c.p.ns);
}

int project_max_chunks(const Ctx& c) {
  int mx = 1;
  for (const BlockDesc& b : c.blocks) mx = std::max(mx, (b.nsupp + kChunk - 1) / kChunk);
  return mx;
}

// Blocks are grouped by their function count; the per-count block lists live
// in the context (built once at bind time).
template <typename T>
void launch_project(const Ctx& c, const T* Y, int ncol, int64_t ld, const T* cscv, const double* coup, T* P,
                    T* Q, hipStream_t st) {
  T* part = reinterpret_cast<T*>(c.d_ppart);
  for (int nm = 1; nm <= kMaxNm; ++nm) {
    const int nblk = c.nm_count[nm];
    if (nblk == 0) continue;
    int maxch = 1;
    for (const BlockDesc& b : c.blocks)
      if (b.nm == nm) maxch = std::max(maxch, (b.nsupp + kChunk - 1) / kChunk);
    const int* d_list = c.d_nm_lists + c.nm_offset[nm];
    switch (nm) {
      case 1: launch_nm<T, 1>(c, Y, ncol, ld, cscv, part, d_list, nblk, maxch, st); break;
      case 2: launch_nm<T, 2>(c, Y, ncol, ld, cscv, part, d_list, nblk, maxch, st); break;
      case 3: launch_nm<T, 3>(c, Y, ncol, ld, cscv, part, d_list, nblk, maxch, st); break;
      case 4: launch_nm<T, 4>(c, Y, ncol, ld, cscv, part, d_list, nblk, maxch, st); break;
      case 5: launch_nm<T, 5>(c, Y, ncol, ld, cscv, part, d_list, nblk, maxch, st); break;
      case 6: launch_nm<T, 6>(c, Y, ncol, ld, cscv, part, d_list, nblk, maxch, st); break;
      case 7: launch_nm<T, 7>(c, Y, ncol, ld, cscv, part, d_list, nblk, maxch, st); break;
      case 8: launch_nm<T, 8>(c, Y, ncol, ld, cscv, part, d_list, nblk, maxch, st); break;
      default: launch_nm<T, 9>(c, Y, ncol, ld, cscv, part, d_list, nblk, maxch, st); break;
    }
  }
  const int nb = (int)c.blocks.size();
  if (nb > 0) {
    dim3 grid((ncol + 63) / 64, nb);
    k_project_finish<T><<<grid, 64, 0, st>>>(part, c.d_blocks, ncol, coup, P, Q, c.nproj, c.p.ns, c.dv);
  }
}

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
}

// Stage 2: P[s][j] = dV * sum of rows jrow[j] .. jrow[j+1] of part (fixed
// order).  One workgroup per (j, 64 states); its 16 waves take every 16th
// row and are combined in a fixed order.
template <typename T>
__global__ __launch_bounds__(1024) void k_slot_sum(const T* __restrict__ part, int ldp, int ncol,
                                                   const int64_t* __restrict__ jrow, T* __restrict__ P, int nproj,
                                                   double dv) {
  __shared__ T red[16][64];
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
    P[(int64_t)s * nproj + j] = (T)dv * x;
  }
}

// Q[j0+m][s] = sum_m' C_b[m][m'] P[s][j0+m'], one thread per (block, state).
template <typename T>
__global__ void k_couple(const T* __restrict__ P, const BlockDesc* __restrict__ blocks, int ncol,
                         const double* __restrict__ coup, T* __restrict__ Q, int nproj, int ldq) {
  const BlockDesc& b = blocks[blockIdx.y];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ncol) return;
  T pv[kMaxNm];
  for (int m = 0; m < b.nm; ++m) pv[m] = P[(int64_t)s * nproj + b.j0 + m];
  const double* cb = coup + b.coup_off;
  for (int m = 0; m < b.nm; ++m) {
    T qv = T(0);
    for (int mp = 0; mp < b.nm; ++mp) qv += (T)cb[m * b.nm + mp] * pv[mp];
    Q[(int64_t)(b.j0 + m) * ldq + s] = qv;
  }
}

size_t project_partial_elems(const Ctx& c) {
  if (c.any_complex || c.pboff.empty()) return 0;
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
  k_proj_brick<T><<<(unsigned)npb * nst, 256, 0, st>>>(Y, ld, ncol, c.d_pboff, c.d_pbnj, (const T*)c.d_pbval[ik],
                                                       c.d_pdest, part, c.p.ns, c.nd, nst, vec);
  dim3 g2((ncol + 63) / 64, c.nproj);
  k_slot_sum<T><<<g2, 1024, 0, st>>>(part, c.p.ns, ncol, c.d_jrow, P, c.nproj, c.dv);
  dim3 g3((ncol + 63) / 64, (unsigned)c.blocks.size());
  k_couple<T><<<g3, 64, 0, st>>>(P, c.d_blocks, ncol, coup, Q, c.nproj, c.p.ns);
}

template void launch_project_brick<double>(const Ctx&, int, const double*, int, int64_t, const double*, double*,
                                           double*, hipStream_t);
template void launch_project_brick<float>(const Ctx&, int, const float*, int, int64_t, const double*, float*,
                                          float*, hipStream_t);

template void launch_project<double>(const Ctx&, const double*, int, int64_t, const double*, const double*,
                                     double*, double*, hipStream_t);
template void launch_project<float>(const Ctx&, const float*, int, int64_t, const float*, const double*, float*,
                                    float*, hipStream_t);
template void launch_project<cplx<double>>(const Ctx&, const cplx<double>*, int, int64_t, const cplx<double>*,
                                           const double*, cplx<double>*, cplx<double>*, hipStream_t);
template void launch_project<cplx<float>>(const Ctx&, const cplx<float>*, int, int64_t, const cplx<float>*,
                                          const double*, cplx<float>*, cplx<float>*, hipStream_t);

}  // namespace hcu
