// Rayleigh-Ritz contractions on the matrix cores (MFMA):
//   S = Y^T Y dV and Hs = Y^T (HY) dV in one pass (split over the grid
//   dimension, deterministic two-stage reduction in FP64), and the subspace
//   rotation X = Y C.  FP64 blocks use v_mfma_f64_16x16x4, FP32 blocks
//   v_mfma_f32_16x16x4 with FP32 accumulation.
//
// Fragment layout of the 16x16x4 MFMA (one wave): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; it receives D[i][l % 16] in
// accumulator element r with i = 4 (l / 16) + r for the FP32 form and
// i = l / 16 + 4 r for the FP64 form (checked on the device).
#include "common.h"

#include <algorithm>
#include <type_traits>

namespace hcu {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct Acc;
template <> struct Acc<double> {
  using V = d4;
  __device__ static inline V mfma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Acc<float> {
  using V = f4;
  __device__ static inline V mfma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int GT = 64;     // output tile (states x states) per workgroup
constexpr int GK = 32;     // grid points per LDS stage
constexpr int GP = GK + 1; // padded LDS row

// part layout: [chunk][tile][2][GT][GT] doubles
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_gram2(const T* __restrict__ Y, const T* __restrict__ HY, int64_t ld,
                                               int n, int64_t nd, int64_t kchunk, const int2* __restrict__ tiles,
                                               int ntiles, double* __restrict__ part) {
  using V = typename Acc<T>::V;
  __shared__ T sA[GT][GP], sB[GT][GP], sH[GT][GP];
  // XCD-contiguous order, tile fastest: the tiles of one grid chunk read the
  // same rows of Y and HY and share them in one L2
  const unsigned lw = xcd_linear();
  const int bx = (int)(lw % gridDim.x), by = (int)(lw / gridDim.x);
  const int2 tl = tiles[bx];
  const int i0 = tl.x * GT, j0 = tl.y * GT;
  const int64_t kb = (int64_t)by * kchunk;
  const int64_t ke = min(nd, kb + kchunk);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  V accS[2][2], accH[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) { accS[a][b][r] = 0; accH[a][b][r] = 0; }
  // the next stage's values are loaded into registers while the current
  // stage is multiplied out of LDS
  constexpr int PER = GT * GK / 256;
  T ra[PER], rb[PER], rh[PER];
  auto fetch = [&](int64_t k) {
    for (int t = 0; t < PER; ++t) {
      const int e = threadIdx.x + 256 * t;
      const int col = e / GK, kk = e % GK;
      const int64_t g = k + kk;
      const bool okk = g < ke;
      ra[t] = (okk && i0 + col < n) ? Y[(int64_t)(i0 + col) * ld + g] : T(0);
      rb[t] = (okk && j0 + col < n) ? Y[(int64_t)(j0 + col) * ld + g] : T(0);
      rh[t] = (okk && j0 + col < n) ? HY[(int64_t)(j0 + col) * ld + g] : T(0);
    }
  };
  if (kb < ke) fetch(kb);
  for (int64_t k = kb; k < ke; k += GK) {
    for (int t = 0; t < PER; ++t) {
      const int e = threadIdx.x + 256 * t;
      const int col = e / GK, kk = e % GK;
      sA[col][kk] = ra[t];
      sB[col][kk] = rb[t];
      sH[col][kk] = rh[t];
    }
    __syncthreads();
    if (k + GK < ke) fetch(k + GK);
    for (int kk = 0; kk < GK; kk += 4) {
      T af[2], bf[2], hf[2];
      for (int a = 0; a < 2; ++a) af[a] = sA[32 * wi + 16 * a + (lane & 15)][kk + (lane >> 4)];
      for (int b = 0; b < 2; ++b) {
        bf[b] = sB[32 * wj + 16 * b + (lane & 15)][kk + (lane >> 4)];
        hf[b] = sH[32 * wj + 16 * b + (lane & 15)][kk + (lane >> 4)];
      }
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          accS[a][b] = Acc<T>::mfma(af[a], bf[b], accS[a][b]);
          accH[a][b] = Acc<T>::mfma(af[a], hf[b], accH[a][b]);
        }
    }
    __syncthreads();
  }
  double* outS = part + ((int64_t)by * ntiles + bx) * 2 * GT * GT;
  double* outH = outS + GT * GT;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) {
        const int i = 32 * wi + 16 * a + Acc<T>::row(lane, r);
        const int j = 32 * wj + 16 * b + (lane & 15);
        outS[i * GT + j] = (double)accS[a][b][r];
        outH[i * GT + j] = (double)accH[a][b][r];
      }
}

// Sum the chunk partials in a fixed order, scale by dV, mirror into full
// symmetric n x n column-major matrices (diagonal tiles symmetrised).
// Grid: (tile, element block of 256, matrix).
__global__ void k_gram_reduce(const double* __restrict__ part, int nchunk, int ntiles,
                              const int2* __restrict__ tiles, int n, double dv, double* __restrict__ S,
                              double* __restrict__ Hs) {
  const int t = blockIdx.x;
  const int w = blockIdx.z;
  const int2 tl = tiles[t];
  const int i0 = tl.x * GT, j0 = tl.y * GT;
  const bool diag = tl.x == tl.y;
  const int e = blockIdx.y * blockDim.x + threadIdx.x;
  if (e >= GT * GT) return;
  const int i = e / GT, j = e % GT;
  if (i0 + i >= n || j0 + j >= n) return;
  if (diag && j < i) return;
  double s1 = 0, s2 = 0;
  const int64_t stride = (int64_t)ntiles * 2 * GT * GT;
  const double* base = part + ((int64_t)t * 2 + w) * GT * GT;
  for (int ch = 0; ch < nchunk; ++ch) {
    s1 += base[ch * stride + i * GT + j];
    if (diag) s2 += base[ch * stride + j * GT + i];
  }
  const double v = diag ? 0.5 * (s1 + s2) * dv : s1 * dv;
  double* M = w == 0 ? S : Hs;
  M[(int64_t)(i0 + i) + (int64_t)(j0 + j) * n] = v;
  M[(int64_t)(j0 + j) + (int64_t)(i0 + i) * n] = v;
}

static void gram_plan(int n, int64_t nd, int& ntiles_1d, int& ntiles, int64_t& kchunk, int& nchunk) {
  ntiles_1d = (n + GT - 1) / GT;
  ntiles = ntiles_1d * (ntiles_1d + 1) / 2;
  int want = std::max(1, 1024 / ntiles);
  kchunk = (nd + want - 1) / want;
  kchunk = ((kchunk + GK - 1) / GK) * GK;
  if (kchunk < 1024) kchunk = 1024;
  nchunk = (int)((nd + kchunk - 1) / kchunk);
}

size_t gram_partial_elems(int n, int64_t nd) {
  int t1, nt, nc;
  int64_t kc;
  gram_plan(n, nd, t1, nt, kc, nc);
  return (size_t)nc * nt * 2 * GT * GT;
}

// Upper-triangular tile list (i <= j) of an n x n Gram matrix, column by
// column: tile t = j (j + 1) / 2 + i.  Every prefix is the list of a smaller
// matrix, so the list built for the context's states serves any ncol <= ns.
std::vector<int2> gram_tiles(int n, bool cplx_) {
  const int t = cplx_ ? 32 : 64;
  const int t1 = (n + t - 1) / t;
  std::vector<int2> tl;
  for (int j = 0; j < t1; ++j)
    for (int i = 0; i <= j; ++i) tl.push_back(make_int2(i, j));
  return tl;
}

// The same list written on the device (no host copy).
__global__ void k_gram_tiles(int2* tiles, int nt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  int j = (int)((sqrt(8.0 * t + 1.0) - 1.0) / 2.0);
  while (j * (j + 1) / 2 > t) --j;
  while ((j + 1) * (j + 2) / 2 <= t) ++j;
  tiles[t] = make_int2(t - j * (j + 1) / 2, j);
}

template <typename T>
void launch_gram2_into(const T* Y, const T* HY, int ncol, int64_t ld, int64_t nd, double dv, const int2* tiles,
                       double* part, double* S, double* Hs, hipStream_t st) {
  int t1, nt, nc;
  int64_t kc;
  gram_plan(ncol, nd, t1, nt, kc, nc);
  launch_k(k_gram2<T>, dim3(nt, nc), 256, 0, st, Y, HY, ld, ncol, nd, kc, tiles, nt, part);
  launch_k(k_gram_reduce, dim3(nt, GT * GT / 256, 2), 256, 0, st, part, nc, nt, tiles, ncol, dv, S, Hs);
}

template <typename T>
void launch_gram2(const Ctx& c, const T* Y, const T* HY, int ncol, int64_t ld, double* S, double* Hs,
                  hipStream_t st) {
  launch_gram2_into<T>(Y, HY, ncol, ld, c.nd, c.dv, c.d_tiles, c.d_part, S, Hs, st);
}

// X = Y C, computed as X^T = C^T Y^T so that each lane's outputs run along the
// grid (contiguous in X).  Workgroup tile: 64 grid points x 64 states.
constexpr int RK = 32;
template <typename T>
__global__ __launch_bounds__(256) void k_rotate(const T* __restrict__ Y, int64_t ld, const T* __restrict__ C,
                                                T* __restrict__ X, int n, int64_t nd) {
  using V = typename Acc<T>::V;
  __shared__ T sY[RK][GT + 1], sC[RK][GT + 1];
  // XCD-contiguous order, state tile fastest: the state tiles of one grid
  // tile read the same rows of Y and share them in one L2
  const unsigned lw = xcd_linear();
  const int j0 = (int)(lw % gridDim.x) * GT;
  const int64_t p0 = (int64_t)(lw / gridDim.x) * GT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wp = wave >> 1, wj = wave & 1;
  V acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) acc[a][b][r] = 0;
  // next stage prefetched into registers during the current stage's products
  constexpr int PER = RK * GT / 256;
  T ry[PER], rc[PER];
  auto fetch = [&](int i0) {
    for (int t = 0; t < PER; ++t) {
      const int e = threadIdx.x + 256 * t;
      const int ii = e / GT, pp = e % GT;
      const int64_t g = p0 + pp;
      ry[t] = (i0 + ii < n && g < nd) ? Y[(int64_t)(i0 + ii) * ld + g] : T(0);
      const int jj = e / RK, i2 = e % RK;
      rc[t] = (i0 + i2 < n && j0 + jj < n) ? C[(int64_t)(j0 + jj) * n + i0 + i2] : T(0);
    }
  };
  fetch(0);
  for (int i0 = 0; i0 < n; i0 += RK) {
    for (int t = 0; t < PER; ++t) {
      const int e = threadIdx.x + 256 * t;
      sY[e / GT][e % GT] = ry[t];
      sC[e % RK][e / RK] = rc[t];
    }
    __syncthreads();
    if (i0 + RK < n) fetch(i0 + RK);
    for (int kk = 0; kk < RK; kk += 4) {
      T af[2], bf[2];
      for (int a = 0; a < 2; ++a) af[a] = sC[kk + (lane >> 4)][32 * wj + 16 * a + (lane & 15)];
      for (int b = 0; b < 2; ++b) bf[b] = sY[kk + (lane >> 4)][32 * wp + 16 * b + (lane & 15)];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = Acc<T>::mfma(af[a], bf[b], acc[a][b]);
    }
    __syncthreads();
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) {
        const int j = j0 + 32 * wj + 16 * a + Acc<T>::row(lane, r);
        const int64_t p = p0 + 32 * wp + 16 * b + (lane & 15);
        if (j < n && p < nd) X[(int64_t)j * ld + p] = acc[a][b][r];
      }
}

// The rotation of real blocks is a plain GEMM, X_c = Y_c C in column-major
// terms (grid points the long dimension): the vendor library's kernel runs it
// faster than k_rotate (c2 FP64 1.24 against 1.58 ms, c3 FP32 6.8 against
// 11.9 ms), so it is used when the context has a library handle; k_rotate
// remains for handle-less calls and the complex kernels below for Bloch
// blocks.
template <typename T>
void launch_rotate(const Ctx& c, const T* Y, int64_t ld, const T* Cb, T* X, int ncol, hipStream_t st) {
  if (c.blas && c.nd <= INT32_MAX && ld <= INT32_MAX) {
    rocblas_set_stream(c.blas, st);
    const T one = T(1), zero = T(0);
    rocblas_status r;
    if constexpr (std::is_same<T, double>::value)
      r = rocblas_dgemm(c.blas, rocblas_operation_none, rocblas_operation_none, (rocblas_int)c.nd, ncol, ncol, &one,
                        Y, (rocblas_int)ld, Cb, ncol, &zero, X, (rocblas_int)ld);
    else
      r = rocblas_sgemm(c.blas, rocblas_operation_none, rocblas_operation_none, (rocblas_int)c.nd, ncol, ncol, &one,
                        Y, (rocblas_int)ld, Cb, ncol, &zero, X, (rocblas_int)ld);
    if (r == rocblas_status_success) return;
  }
  dim3 grid((ncol + GT - 1) / GT, (unsigned)((c.nd + GT - 1) / GT));
  launch_k(k_rotate<T>, grid, 256, 0, st, Y, ld, Cb, X, ncol, c.nd);
}

// PX[s][j] = sum_i C[i][s] PY[i][j]  (projections follow the rotation)
template <typename T>
__global__ void k_rotate_proj(const T* __restrict__ PY, const T* __restrict__ C, T* __restrict__ PX, int n,
                              int nproj) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (j >= nproj) return;
  T acc = T(0);
  for (int i = 0; i < n; ++i) acc += C[(int64_t)s * n + i] * PY[(int64_t)i * nproj + j];
  PX[(int64_t)s * nproj + j] = acc;
}

template <typename T>
void launch_rotate_proj(const Ctx& c, const T* PY, const T* Cb, T* PX, int ncol, hipStream_t st) {
  if (c.nproj == 0) return;
  dim3 grid((c.nproj + 127) / 128, ncol);
  launch_k(k_rotate_proj<T>, grid, 128, 0, st, PY, Cb, PX, ncol, c.nproj);
}

template void launch_gram2<double>(const Ctx&, const double*, const double*, int, int64_t, double*, double*, hipStream_t);
template void launch_gram2<float>(const Ctx&, const float*, const float*, int, int64_t, double*, double*, hipStream_t);
template void launch_rotate<double>(const Ctx&, const double*, int64_t, const double*, double*, int, hipStream_t);
template void launch_rotate<float>(const Ctx&, const float*, int64_t, const float*, float*, int, hipStream_t);
template void launch_rotate_proj<double>(const Ctx&, const double*, const double*, double*, int, hipStream_t);
template void launch_rotate_proj<float>(const Ctx&, const float*, const float*, float*, int, hipStream_t);

// ---------------------------------------------------------------- complex blocks
// Complex (Bloch) blocks: S = Y^H Y dV, Hs = Y^H HY dV (Hermitian), X = Y C;
// complex FP32 on the matrix cores (k_gram2_cm, k_rotate_cm), complex FP64
// on VALU tiles.  Partials hold interleaved complex doubles.
constexpr int CT = 32;     // output tile
constexpr int CK = 32;     // grid points per stage
template <typename T>
__global__ __launch_bounds__(256) void k_gram2_c(const T* __restrict__ Y, const T* __restrict__ HY, int64_t ld,
                                                 int n, int64_t nd, int64_t kchunk, const int2* __restrict__ tiles,
                                                 int ntiles, double* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) unsigned char raw[3 * CT * (CK + 1) * sizeof(T)];
  T(*sA)[CK + 1] = reinterpret_cast<T(*)[CK + 1]>(raw);
  T(*sB)[CK + 1] = sA + CT;
  T(*sH)[CK + 1] = sB + CT;
  // XCD-contiguous order, tile fastest: the tiles of one grid chunk read the
  // same rows of Y and HY and share them in one L2
  const unsigned lw = xcd_linear();
  const int bx = (int)(lw % gridDim.x), by = (int)(lw / gridDim.x);
  const int2 tl = tiles[bx];
  const int i0 = tl.x * CT, j0 = tl.y * CT;
  const int64_t kb = (int64_t)by * kchunk;
  const int64_t ke = min(nd, kb + kchunk);
  const int ti = threadIdx.x / 8, tj = (threadIdx.x % 8) * 4;
  T aS[4], aH[4];
  for (int q = 0; q < 4; ++q) { aS[q] = T(0); aH[q] = T(0); }
  for (int64_t k = kb; k < ke; k += CK) {
    for (int e = threadIdx.x; e < CT * CK; e += 256) {
      const int col = e / CK, kk = e % CK;
      const int64_t g = k + kk;
      const bool okk = g < ke;
      sA[col][kk] = (okk && i0 + col < n) ? Y[(int64_t)(i0 + col) * ld + g] : T(0);
      sB[col][kk] = (okk && j0 + col < n) ? Y[(int64_t)(j0 + col) * ld + g] : T(0);
      sH[col][kk] = (okk && j0 + col < n) ? HY[(int64_t)(j0 + col) * ld + g] : T(0);
    }
    __syncthreads();
    for (int kk = 0; kk < CK; ++kk) {
      const T a = conj_(sA[ti][kk]);
      for (int q = 0; q < 4; ++q) {
        aS[q] += a * sB[tj + q][kk];
        aH[q] += a * sH[tj + q][kk];
      }
    }
    __syncthreads();
  }
  double* outS = part + ((int64_t)by * ntiles + bx) * 2 * CT * CT * 2;
  double* outH = outS + CT * CT * 2;
  for (int q = 0; q < 4; ++q) {
    const int e = ti * CT + tj + q;
    outS[2 * e] = (double)aS[q].re; outS[2 * e + 1] = (double)aS[q].im;
    outH[2 * e] = (double)aH[q].re; outH[2 * e + 1] = (double)aH[q].im;
  }
}

// Complex FP32 blocks on the matrix cores: the same 32 x 32 output tiles and
// partial layout as k_gram2_c, each wave one 16 x 16 sub-tile of S and of Hs,
// each complex product as three real ones (Gauss) in separate accumulators:
// for A^H B, Re = Σ ar br + Σ ai bi, Im = Σ (ar - ai)(br + bi) - Σ ar br +
// Σ ai bi; staged through LDS as separate real and imaginary planes, next
// stage prefetched into registers from clamped in-range addresses (zeroed by
// selection when staged: a guarded load would wait for every outstanding one).
template <typename R>
__global__ __launch_bounds__(256) void k_gram2_cm(const cplx<R>* __restrict__ Y, const cplx<R>* __restrict__ HY,
                                                  int64_t ld, int n, int64_t nd, int64_t kchunk,
                                                  const int2* __restrict__ tiles, int ntiles,
                                                  double* __restrict__ part) {
  using V = typename Acc<R>::V;
  using C = cplx<R>;
  __shared__ R sAr[CT][CK + 1], sAi[CT][CK + 1], sBr[CT][CK + 1], sBi[CT][CK + 1], sHr[CT][CK + 1],
      sHi[CT][CK + 1];
  // XCD-contiguous order, tile fastest: the tiles of one grid chunk read the
  // same rows of Y and HY and share them in one L2
  const unsigned lw = xcd_linear();
  const int bx = (int)(lw % gridDim.x), by = (int)(lw / gridDim.x);
  const int2 tl = tiles[bx];
  const int i0 = tl.x * CT, j0 = tl.y * CT;
  const int64_t kb = (int64_t)by * kchunk;
  const int64_t ke = min(nd, kb + kchunk);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  V acc[6];   // S: rr ii (r-i)(r+i), Hs: rr ii (r-i)(r+i)
  for (int t = 0; t < 6; ++t)
    for (int r = 0; r < 4; ++r) acc[t][r] = 0;
  constexpr int PER = CT * CK / 256;
  C ra[PER], rb[PER], rh[PER];
  auto fetch = [&](int64_t k) {   // k < ke
    for (int t = 0; t < PER; ++t) {
      const int e = threadIdx.x + 256 * t;
      const int col = e / CK, kk = e % CK;
      const int64_t g = min(k + kk, ke - 1);
      const int ca = min(i0 + col, n - 1), cb = min(j0 + col, n - 1);
      ra[t] = Y[(int64_t)ca * ld + g];
      rb[t] = Y[(int64_t)cb * ld + g];
      rh[t] = HY[(int64_t)cb * ld + g];
    }
  };
  if (kb < ke) fetch(kb);
  for (int64_t k = kb; k < ke; k += CK) {
    for (int t = 0; t < PER; ++t) {
      const int e = threadIdx.x + 256 * t;
      const int col = e / CK, kk = e % CK;
      const bool okk = k + kk < ke;
      const bool oa = okk && i0 + col < n, ob = okk && j0 + col < n;
      sAr[col][kk] = oa ? ra[t].re : R(0);
      sAi[col][kk] = oa ? ra[t].im : R(0);
      sBr[col][kk] = ob ? rb[t].re : R(0);
      sBi[col][kk] = ob ? rb[t].im : R(0);
      sHr[col][kk] = ob ? rh[t].re : R(0);
      sHi[col][kk] = ob ? rh[t].im : R(0);
    }
    __syncthreads();
    if (k + CK < ke) fetch(k + CK);
    for (int kk = 0; kk < CK; kk += 4) {
      const int ia = 16 * wi + (lane & 15), jb = 16 * wj + (lane & 15), kq = kk + (lane >> 4);
      const R ar = sAr[ia][kq], ai = sAi[ia][kq];
      const R br = sBr[jb][kq], bi = sBi[jb][kq], hr = sHr[jb][kq], hi = sHi[jb][kq];
      const R ad = ar - ai;
      acc[0] = Acc<R>::mfma(ar, br, acc[0]);
      acc[1] = Acc<R>::mfma(ai, bi, acc[1]);
      acc[2] = Acc<R>::mfma(ad, br + bi, acc[2]);
      acc[3] = Acc<R>::mfma(ar, hr, acc[3]);
      acc[4] = Acc<R>::mfma(ai, hi, acc[4]);
      acc[5] = Acc<R>::mfma(ad, hr + hi, acc[5]);
    }
    __syncthreads();
  }
  double* outS = part + ((int64_t)by * ntiles + bx) * 2 * CT * CT * 2;
  double* outH = outS + CT * CT * 2;
  for (int r = 0; r < 4; ++r) {
    const int i = 16 * wi + Acc<R>::row(lane, r);
    const int j = 16 * wj + (lane & 15);
    const int e = i * CT + j;
    outS[2 * e] = (double)acc[0][r] + (double)acc[1][r];
    outS[2 * e + 1] = (double)acc[2][r] - (double)acc[0][r] + (double)acc[1][r];
    outH[2 * e] = (double)acc[3][r] + (double)acc[4][r];
    outH[2 * e + 1] = (double)acc[5][r] - (double)acc[3][r] + (double)acc[4][r];
  }
}

__global__ void k_gram_reduce_c(const double* __restrict__ part, int nchunk, int ntiles,
                                const int2* __restrict__ tiles, int n, double dv, double* __restrict__ S,
                                double* __restrict__ Hs) {
  const int t = blockIdx.x;
  const int2 tl = tiles[t];
  const int i0 = tl.x * CT, j0 = tl.y * CT;
  const bool diag = tl.x == tl.y;
  for (int e = threadIdx.x; e < CT * CT; e += blockDim.x) {
    const int i = e / CT, j = e % CT;
    if (i0 + i >= n || j0 + j >= n) continue;
    if (diag && j < i) continue;
    for (int w = 0; w < 2; ++w) {
      double r1 = 0, m1 = 0, r2 = 0, m2 = 0;
      for (int ch = 0; ch < nchunk; ++ch) {
        const double* base = part + (((int64_t)ch * ntiles + t) * 2 + w) * CT * CT * 2;
        r1 += base[2 * (i * CT + j)];
        m1 += base[2 * (i * CT + j) + 1];
        if (diag) { r2 += base[2 * (j * CT + i)]; m2 += base[2 * (j * CT + i) + 1]; }
      }
      double re = diag ? 0.5 * (r1 + r2) : r1, im = diag ? 0.5 * (m1 - m2) : m1;
      re *= dv; im *= dv;
      double* M = w == 0 ? S : Hs;
      const int64_t a = (int64_t)(i0 + i) + (int64_t)(j0 + j) * n, b = (int64_t)(j0 + j) + (int64_t)(i0 + i) * n;
      M[2 * a] = re; M[2 * a + 1] = im;
      M[2 * b] = re; M[2 * b + 1] = -im;
    }
  }
}

static void gram_plan_c(int n, int64_t nd, int& t1, int& nt, int64_t& kchunk, int& nchunk) {
  t1 = (n + CT - 1) / CT;
  nt = t1 * (t1 + 1) / 2;
  int want = std::max(1, 2048 / nt);
  kchunk = (nd + want - 1) / want;
  kchunk = ((kchunk + CK - 1) / CK) * CK;
  if (kchunk < 1024) kchunk = 1024;
  nchunk = (int)((nd + kchunk - 1) / kchunk);
}

size_t gram_partial_elems_c(int n, int64_t nd) {
  int t1, nt, nc;
  int64_t kc;
  gram_plan_c(n, nd, t1, nt, kc, nc);
  return (size_t)nc * nt * 2 * CT * CT * 2;
}

template <typename T>
void launch_gram2_c_into(const T* Y, const T* HY, int ncol, int64_t ld, int64_t nd, double dv, const int2* tiles,
                         double* part, double* S, double* Hs, hipStream_t st) {
  int t1, nt, nc;
  int64_t kc;
  gram_plan_c(ncol, nd, t1, nt, kc, nc);
  if constexpr (std::is_same<T, cplx<float>>::value)
    launch_k(k_gram2_cm<float>, dim3(nt, nc), 256, 0, st, Y, HY, ld, ncol, nd, kc, tiles, nt, part);
  else
    launch_k(k_gram2_c<T>, dim3(nt, nc), 256, 0, st, Y, HY, ld, ncol, nd, kc, tiles, nt, part);
  launch_k(k_gram_reduce_c, nt, 256, 0, st, part, nc, nt, tiles, ncol, dv, S, Hs);
}

template <typename T>
void launch_gram2_c(const Ctx& c, const T* Y, const T* HY, int ncol, int64_t ld, double* S, double* Hs,
                    hipStream_t st) {
  launch_gram2_c_into<T>(Y, HY, ncol, ld, c.nd, c.dv, c.d_tiles, c.d_part, S, Hs, st);
}

// X = Y C for complex blocks: workgroup = 64 grid points x 32 states.
template <typename T>
__global__ __launch_bounds__(256) void k_rotate_c(const T* __restrict__ Y, int64_t ld, const T* __restrict__ C,
                                                  T* __restrict__ X, int n, int64_t nd) {
  __shared__ __attribute__((aligned(16))) unsigned char raw[(16 * 64 + 16 * CT) * sizeof(T)];
  T(*sY)[64] = reinterpret_cast<T(*)[64]>(raw);
  T(*sC)[CT] = reinterpret_cast<T(*)[CT]>(raw + 16 * 64 * sizeof(T));
  // XCD-contiguous order, state tile fastest: the state tiles of one grid
  // tile read the same rows of Y and share them in one L2
  const unsigned lw = xcd_linear();
  const int j0 = (int)(lw % gridDim.x) * CT;
  const int64_t p0 = (int64_t)(lw / gridDim.x) * 64;
  const int tp = threadIdx.x % 64, tj = (threadIdx.x / 64) * 8;
  T acc[8];
  for (int q = 0; q < 8; ++q) acc[q] = T(0);
  for (int i0 = 0; i0 < n; i0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int ii = e / 64, pp = e % 64;
      sY[ii][pp] = (i0 + ii < n && p0 + pp < nd) ? Y[(int64_t)(i0 + ii) * ld + p0 + pp] : T(0);
    }
    for (int e = threadIdx.x; e < 16 * CT; e += 256) {
      const int jj = e / 16, ii = e % 16;
      sC[ii][jj] = (i0 + ii < n && j0 + jj < n) ? C[(int64_t)(j0 + jj) * n + i0 + ii] : T(0);
    }
    __syncthreads();
    for (int ii = 0; ii < 16; ++ii) {
      const T y = sY[ii][tp];
      for (int q = 0; q < 8; ++q) acc[q] += y * sC[ii][tj + q];
    }
    __syncthreads();
  }
  for (int q = 0; q < 8; ++q) {
    const int j = j0 + tj + q;
    if (j < n && p0 + tp < nd) X[(int64_t)j * ld + p0 + tp] = acc[q];
  }
}

// Complex FP32 rotation on the matrix cores: X^T = C^T Y^T as in k_rotate
// (64 states x 64 grid points per workgroup, each wave 2 x 2 sub-tiles), the
// complex product as four real ones: Re X = rr - ii, Im X = ir + ri
// (first letter C, second Y).
template <typename R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_rotate_cm(
    const cplx<R>* __restrict__ Y, int64_t ld, const cplx<R>* __restrict__ Cm, cplx<R>* __restrict__ X, int n,
    int64_t nd) {
  using V = typename Acc<R>::V;
  using C = cplx<R>;
  __shared__ R sYr[RK][GT + 1], sYi[RK][GT + 1], sCr[RK][GT + 1], sCi[RK][GT + 1];
  // XCD-contiguous order, state tile fastest: the state tiles of one grid
  // tile read the same rows of Y and share them in one L2
  const unsigned lw = xcd_linear();
  const int j0 = (int)(lw % gridDim.x) * GT;
  const int64_t p0 = (int64_t)(lw / gridDim.x) * GT;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wp = wave >> 1, wj = wave & 1;
  V acc[2][2][4];   // rr ii ir ri
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int h = 0; h < 4; ++h)
        for (int r = 0; r < 4; ++r) acc[a][b][h][r] = 0;
  constexpr int PER = RK * GT / 256;
  C ry[PER], rc[PER];
  auto fetch = [&](int i0) {
    for (int t = 0; t < PER; ++t) {
      const int e = threadIdx.x + 256 * t;
      const int ii = e / GT, pp = e % GT;
      const int64_t g = p0 + pp;
      ry[t] = (i0 + ii < n && g < nd) ? Y[(int64_t)(i0 + ii) * ld + g] : C();
      const int jj = e / RK, i2 = e % RK;
      rc[t] = (i0 + i2 < n && j0 + jj < n) ? Cm[(int64_t)(j0 + jj) * n + i0 + i2] : C();
    }
  };
  fetch(0);
  for (int i0 = 0; i0 < n; i0 += RK) {
    for (int t = 0; t < PER; ++t) {
      const int e = threadIdx.x + 256 * t;
      sYr[e / GT][e % GT] = ry[t].re;
      sYi[e / GT][e % GT] = ry[t].im;
      sCr[e % RK][e / RK] = rc[t].re;
      sCi[e % RK][e / RK] = rc[t].im;
    }
    __syncthreads();
    if (i0 + RK < n) fetch(i0 + RK);
    for (int kk = 0; kk < RK; kk += 4) {
      R cr[2], ci[2], yr[2], yi[2];
      for (int a = 0; a < 2; ++a) {
        cr[a] = sCr[kk + (lane >> 4)][32 * wj + 16 * a + (lane & 15)];
        ci[a] = sCi[kk + (lane >> 4)][32 * wj + 16 * a + (lane & 15)];
      }
      for (int b = 0; b < 2; ++b) {
        yr[b] = sYr[kk + (lane >> 4)][32 * wp + 16 * b + (lane & 15)];
        yi[b] = sYi[kk + (lane >> 4)][32 * wp + 16 * b + (lane & 15)];
      }
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          acc[a][b][0] = Acc<R>::mfma(cr[a], yr[b], acc[a][b][0]);
          acc[a][b][1] = Acc<R>::mfma(ci[a], yi[b], acc[a][b][1]);
          acc[a][b][2] = Acc<R>::mfma(ci[a], yr[b], acc[a][b][2]);
          acc[a][b][3] = Acc<R>::mfma(cr[a], yi[b], acc[a][b][3]);
        }
    }
    __syncthreads();
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) {
        const int j = j0 + 32 * wj + 16 * a + Acc<R>::row(lane, r);
        const int64_t p = p0 + 32 * wp + 16 * b + (lane & 15);
        if (j < n && p < nd)
          X[(int64_t)j * ld + p] = C(acc[a][b][0][r] - acc[a][b][1][r], acc[a][b][2][r] + acc[a][b][3][r]);
      }
}

template <typename T>
void launch_rotate_c(const Ctx& c, const T* Y, int64_t ld, const T* Cb, T* X, int ncol, hipStream_t st) {
  // X_c = Y_c C (no conjugation) as a plain complex GEMM through the vendor
  // library, as for real blocks; the kernels below without a handle
  if (c.blas && c.nd <= INT32_MAX && ld <= INT32_MAX) {
    rocblas_set_stream(c.blas, st);
    rocblas_status r;
    if constexpr (std::is_same<T, cplx<float>>::value) {
      using B = rocblas_float_complex;
      const B one{1.0f, 0.0f}, zero{0.0f, 0.0f};
      r = rocblas_cgemm(c.blas, rocblas_operation_none, rocblas_operation_none, (rocblas_int)c.nd, ncol, ncol, &one,
                        reinterpret_cast<const B*>(Y), (rocblas_int)ld, reinterpret_cast<const B*>(Cb), ncol, &zero,
                        reinterpret_cast<B*>(X), (rocblas_int)ld);
    } else {
      using B = rocblas_double_complex;
      const B one{1.0, 0.0}, zero{0.0, 0.0};
      r = rocblas_zgemm(c.blas, rocblas_operation_none, rocblas_operation_none, (rocblas_int)c.nd, ncol, ncol, &one,
                        reinterpret_cast<const B*>(Y), (rocblas_int)ld, reinterpret_cast<const B*>(Cb), ncol, &zero,
                        reinterpret_cast<B*>(X), (rocblas_int)ld);
    }
    if (r == rocblas_status_success) return;
  }
  if constexpr (std::is_same<T, cplx<float>>::value) {
    dim3 grid((ncol + GT - 1) / GT, (unsigned)((c.nd + GT - 1) / GT));
    launch_k(k_rotate_cm<float>, grid, 256, 0, st, Y, ld, Cb, X, ncol, c.nd);
  } else {
    dim3 grid((ncol + CT - 1) / CT, (unsigned)((c.nd + 63) / 64));
    launch_k(k_rotate_c<T>, grid, 256, 0, st, Y, ld, Cb, X, ncol, c.nd);
  }
}

template <>
void launch_gram2<cplx<double>>(const Ctx& c, const cplx<double>* Y, const cplx<double>* HY, int ncol, int64_t ld,
                                double* S, double* Hs, hipStream_t st) {
  launch_gram2_c(c, Y, HY, ncol, ld, S, Hs, st);
}
template <>
void launch_gram2<cplx<float>>(const Ctx& c, const cplx<float>* Y, const cplx<float>* HY, int ncol, int64_t ld,
                               double* S, double* Hs, hipStream_t st) {
  launch_gram2_c(c, Y, HY, ncol, ld, S, Hs, st);
}
template <>
void launch_rotate<cplx<double>>(const Ctx& c, const cplx<double>* Y, int64_t ld, const cplx<double>* Cb,
                                 cplx<double>* X, int ncol, hipStream_t st) {
  launch_rotate_c(c, Y, ld, Cb, X, ncol, st);
}
template <>
void launch_rotate<cplx<float>>(const Ctx& c, const cplx<float>* Y, int64_t ld, const cplx<float>* Cb,
                                cplx<float>* X, int ncol, hipStream_t st) {
  launch_rotate_c(c, Y, ld, Cb, X, ncol, st);
}
// Gram contractions with caller-given scratch (partials and tile list): the
// tile list is written on the device first, then the contraction and its
// reduction run as in launch_gram2.
static int gram_ntiles(int ncol, bool cplx_) {
  const int t = cplx_ ? CT : GT;
  const int t1 = (ncol + t - 1) / t;
  return t1 * (t1 + 1) / 2;
}

size_t gram_scratch_bytes(int ncol, int64_t nd, bool cplx_) {
  const size_t part = sizeof(double) * (cplx_ ? gram_partial_elems_c(ncol, nd) : gram_partial_elems(ncol, nd));
  return ((part + 255) & ~size_t(255)) + sizeof(int2) * (size_t)gram_ntiles(ncol, cplx_);
}

void launch_gram_scratch(const void* Y, const void* HY, int ncol, int64_t ld, int64_t nd, double dv, bool fp32,
                         bool cplx_, void* scratch, double* S, double* Hs, hipStream_t st) {
  const size_t part_bytes = sizeof(double) * (cplx_ ? gram_partial_elems_c(ncol, nd) : gram_partial_elems(ncol, nd));
  double* part = reinterpret_cast<double*>(scratch);
  int2* tiles = reinterpret_cast<int2*>(reinterpret_cast<char*>(scratch) + ((part_bytes + 255) & ~size_t(255)));
  const int nt = gram_ntiles(ncol, cplx_);
  launch_k(k_gram_tiles, (nt + 255) / 256, 256, 0, st, tiles, nt);
  if (!cplx_) {
    if (fp32)
      launch_gram2_into<float>((const float*)Y, (const float*)HY, ncol, ld, nd, dv, tiles, part, S, Hs, st);
    else
      launch_gram2_into<double>((const double*)Y, (const double*)HY, ncol, ld, nd, dv, tiles, part, S, Hs, st);
  } else {
    if (fp32)
      launch_gram2_c_into<cplx<float>>((const cplx<float>*)Y, (const cplx<float>*)HY, ncol, ld, nd, dv, tiles, part,
                                       S, Hs, st);
    else
      launch_gram2_c_into<cplx<double>>((const cplx<double>*)Y, (const cplx<double>*)HY, ncol, ld, nd, dv, tiles,
                                        part, S, Hs, st);
  }
}

template void launch_rotate_proj<cplx<double>>(const Ctx&, const cplx<double>*, const cplx<double>*, cplx<double>*,
                                               int, hipStream_t);
template void launch_rotate_proj<cplx<float>>(const Ctx&, const cplx<float>*, const cplx<float>*, cplx<float>*, int,
                                              hipStream_t);

}  // namespace hcu
