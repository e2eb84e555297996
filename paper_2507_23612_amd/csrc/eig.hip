// Dense symmetric eigensolve of the Rayleigh-Ritz step (Sec. II.B: the
// projected problem of Chebyshev-filtered subspace iteration): Householder
// reduction to tridiagonal form in ONE workgroup.
//
// The library's blocked reduction issues a chain of small kernels per column
// (matrix-vector product, reflector, dot products): at the Rayleigh-Ritz
// sizes (N_s of a few hundred) it is bound by launch latency, not by work.
// Here one workgroup of 1024 threads keeps the active block in the L2 of its
// XCD (512 KB at N = 256) and performs every column in place:
//
//   for i = n-2 .. 0 (column i+1, entries 0..i):
//     reflector H_i = I - tau v v^T with v(i) = 1 annihilating A(0:i-1, i+1)
//     (beta = -sign(alpha) |(alpha, x)|, tau = (beta - alpha)/beta,
//      v(0:i-1) = x / (alpha - beta); tau = 0 when x = 0)
//     p = A(0:i, 0:i) v,  w = tau p - (tau^2 / 2)(p . v) v
//     A(0:i, 0:i) -= v w^T + w v^T
//
// with the storage of the standard upper-triangle reduction (v of H_i in
// A(0:i-1, i+1), T's superdiagonal in A(i, i+1) and e, its diagonal in d,
// tau in tau), so the library's tridiagonal divide-and-conquer and its
// back-transformation by the reflectors apply unchanged.  The rank-2 update
// of step i is fused with the matrix-vector product of step i-1: column i
// is updated first, it yields the next reflector, and one sweep over the
// remaining block then writes A - v w^T - w v^T and accumulates A_new v'.
// Each element is read and written once per column.
#include "common.h"

namespace hcu {
namespace {

constexpr int kTdThreads = 1024;
constexpr int kTdWaves = kTdThreads / 64;
constexpr int kTdMaxN = 512;
constexpr int kTdUnroll = 8;

__device__ inline double td_block_sum(double x, double* red) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
  __syncthreads();
  double s = 0;
  for (int i = 0; i < kTdWaves; ++i) s += red[i];
  return s;
}

// One sweep over the block (r, c) in [0, m)^2:
//   upd: A(r, c) -= v_r w_c + w_r v_c (written back), then
//   p_r = sum_c A(r, c) vn_c  (the next step's matrix-vector product).
// Wave layout: nrb = ceil(m / 64) row blocks of 64 rows (one row per lane),
// g = 16 / nrb column groups; wave (rb, cg) takes columns cg, cg + g, ...
// Partial sums per wave go through LDS (part[wave][lane]) and are summed in
// a fixed order.
__device__ void td_sweep(double* __restrict__ A, int lda, int m, bool upd, const double* v, const double* w,
                         const double* vn, double* part, double* p) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nrb = (m + 63) >> 6;
  const int g = kTdWaves / nrb;
  const int rb = wv % nrb, cg = wv / nrb;
  const int r = 64 * rb + lane;
  double acc = 0;
  if (cg < g && r < m) {
    const double vr = v[r], wr = w[r];
    double* col = A + r;
    int c = cg;
    for (; c + (kTdUnroll - 1) * g < m; c += kTdUnroll * g) {
      double a[kTdUnroll];
#pragma unroll
      for (int u = 0; u < kTdUnroll; ++u) a[u] = col[(int64_t)(c + u * g) * lda];
#pragma unroll
      for (int u = 0; u < kTdUnroll; ++u) {
        const int cc = c + u * g;
        if (upd) {
          a[u] -= vr * w[cc] + wr * v[cc];
          col[(int64_t)cc * lda] = a[u];
        }
        acc += a[u] * vn[cc];
      }
    }
    for (; c < m; c += g) {
      double a = col[(int64_t)c * lda];
      if (upd) {
        a -= vr * w[c] + wr * v[c];
        col[(int64_t)c * lda] = a;
      }
      acc += a * vn[c];
    }
  }
  part[wv * 64 + lane] = acc;
  __syncthreads();
  if (threadIdx.x < m) {
    const int rr = threadIdx.x, b = rr >> 6, l = rr & 63;
    double s = 0;
    for (int k = 0; k < g; ++k) s += part[(k * nrb + b) * 64 + l];
    p[rr] = s;
  }
  __syncthreads();
}

// Reflector of column c from the values x_r (r < len) held by threads r:
// alpha = x_{len-1}, the rest is annihilated.  Writes v (v[len-1] = 1), the
// scaled entries back to A(0:len-2, c) and beta to A(len-1, c); returns tau
// and beta through sc.
__device__ void td_reflector(double* __restrict__ A, int lda, int c, int len, double xr, double* vout,
                             double* red, double* sc) {
  const int t = threadIdx.x;
  const double s2 = td_block_sum(t < len - 1 ? xr * xr : 0.0, red);
  if (t == len - 1) sc[2] = xr;   // alpha
  __syncthreads();
  const double alpha = sc[2];
  double tau = 0.0, beta = alpha, scale = 1.0;
  if (s2 > 0.0) {
    const double nrm = sqrt(alpha * alpha + s2);
    beta = alpha >= 0.0 ? -nrm : nrm;
    tau = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  if (t < len - 1) {
    const double x = tau != 0.0 ? xr * scale : xr;
    A[t + (int64_t)c * lda] = x;
    vout[t] = x;
  } else if (t == len - 1) {
    A[t + (int64_t)c * lda] = beta;
    vout[t] = 1.0;
  }
  if (t == 0) { sc[0] = tau; sc[1] = beta; }
  __syncthreads();
}

__global__ __launch_bounds__(kTdThreads) void k_sytrd_small(double* __restrict__ A, int n, int lda,
                                                            double* __restrict__ d, double* __restrict__ e,
                                                            double* __restrict__ taus) {
  __shared__ double v[kTdMaxN], w[kTdMaxN], vn[kTdMaxN], p[kTdMaxN];
  __shared__ double part[kTdThreads];
  __shared__ double red[kTdWaves];
  __shared__ double sc[4];
  const int t = threadIdx.x;
  // the lower triangle from the upper one (the reduction reads full columns)
  for (int64_t q = t; q < (int64_t)n * n; q += kTdThreads) {
    const int r = (int)(q % n), c = (int)(q / n);
    if (r > c) A[r + (int64_t)c * lda] = A[c + (int64_t)r * lda];
  }
  __syncthreads();
  if (t == 0) d[n - 1] = A[(n - 1) + (int64_t)(n - 1) * lda];
  if (n == 1) return;
  // first reflector (column n-1) and its matrix-vector product
  {
    const int len = n - 1;
    const double x = t < len ? A[t + (int64_t)(n - 1) * lda] : 0.0;
    td_reflector(A, lda, n - 1, len, x, v, red, sc);
    td_sweep(A, lda, len, false, v, v, v, part, p);
  }
  for (int i = n - 2; i >= 0; --i) {
    // v, p = A(0:i,0:i) v and tau of step i are ready
    const double tau = sc[0], beta = sc[1];
    const double wi = t <= i ? tau * p[t] : 0.0;
    const double dot = td_block_sum(t <= i ? wi * v[t] : 0.0, red);
    const double a2 = -0.5 * tau * dot;
    if (t <= i) w[t] = wi + a2 * v[t];
    if (t == 0) { e[i] = beta; taus[i] = tau; }
    __syncthreads();
    if (i == 0) {
      if (t == 0) d[0] = A[0] - 2.0 * v[0] * w[0];
      break;
    }
    // column i of the updated block (entries r < i) and its diagonal
    double xr = 0.0;
    if (t < i) xr = A[t + (int64_t)i * lda] - (v[t] * w[i] + w[t] * v[i]);
    if (t == i) d[i] = A[i + (int64_t)i * lda] - 2.0 * v[i] * w[i];
    // next reflector from column i (length i), then the fused sweep over [0, i)^2
    td_reflector(A, lda, i, i, xr, vn, red, sc);
    td_sweep(A, lda, i, tau != 0.0, v, w, vn, part, p);
    if (t < i) v[t] = vn[t];
    __syncthreads();
  }
}

// ---------------------------------------------------------------- n <= 256
// The same reduction with the upper triangle held in registers: 8 waves;
// wave w owns the columns c = w + 8 j (j < 32), lane l holds rows
// r = 64 k + l (k <= j / 8, rows up to the column's diagonal) of each of
// them, 80 doubles per lane (two waves per SIMD, 256 registers each),
// always indexed with compile-time constants.
// Nothing but the finished reflector columns is written to memory.  Each
// sweep also leaves the column the next step starts from (c = m - 1) in LDS,
// where the reflector is formed by the whole workgroup.  The matrix-vector
// product accumulates a column-wise part (sum over r of A(r, c) vn_r,
// reduced across the owner wave into pc[c]) and a row-wise part (the
// mirrored lower triangle, A(r, c) vn_c for r < c, per lane, then across
// the waves in a fixed order).
constexpr int kRgWaves = 8;
constexpr int kRgThreads = 64 * kRgWaves;
constexpr int kRgCols = 32;                  // columns per wave
constexpr int kRgMaxN = kRgWaves * kRgCols;  // 256
constexpr int kRgChunks = 4;                 // 64-row chunks of the longest column

// 64-row chunks of the wave's j-th column (its largest index is 8 j + 7)
__host__ __device__ constexpr int rg_nch(int j) { return (kRgWaves * j + kRgWaves - 1) / 64 + 1; }
__host__ __device__ constexpr int rg_off(int j) { return j <= 0 ? 0 : rg_off(j - 1) + rg_nch(j - 1); }
constexpr int kRgRegs = rg_off(kRgCols);     // 80

// Data-parallel-primitive move of a double (each 32-bit half moved by the
// same DPP control; lanes whose source is outside the row, or whose row is
// masked off, receive 0).
template <int CTRL, int ROWS>
__device__ inline double dpp_mov(double x) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, ROWS, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Sum over the 64 lanes of a wave, valid in lane 63: inclusive scans inside
// each 16-lane row (row shifts by 1, 2, 4, 8), then the row totals carried
// across rows (row broadcasts of lanes 15 and 31).  All VALU moves, no LDS
// crossbar round trips.
__device__ inline double wave_sum_lane63(double x) {
  x += dpp_mov<0x111, 0xf>(x);   // row_shr:1
  x += dpp_mov<0x112, 0xf>(x);   // row_shr:2
  x += dpp_mov<0x114, 0xf>(x);   // row_shr:4
  x += dpp_mov<0x118, 0xf>(x);   // row_shr:8
  x += dpp_mov<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
  x += dpp_mov<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3
  return x;
}

__global__ __launch_bounds__(kRgThreads) void k_sytrd_reg(double* __restrict__ A, int n, int lda,
                                                          double* __restrict__ d, double* __restrict__ e,
                                                          double* __restrict__ taus) {
  __shared__ double v[kRgMaxN], w[kRgMaxN], vn[kRgMaxN], pc[kRgMaxN], colbuf[kRgMaxN];
  __shared__ double part[kRgWaves * kRgChunks * 64];
  __shared__ double red[kRgWaves];
  __shared__ double sc[4];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  double a[kRgRegs];
#pragma unroll
  for (int j = 0; j < kRgCols; ++j) {
    const int c = wv + kRgWaves * j;
#pragma unroll
    for (int k = 0; k < rg_nch(j); ++k) {
      const int r = 64 * k + lane;
      a[rg_off(j) + k] = (c < n && r <= c) ? A[r + (int64_t)c * lda] : 0.0;
    }
  }
  if (t < kRgMaxN) {
    v[t] = 0.0;
    w[t] = 0.0;
    vn[t] = 0.0;
    colbuf[t] = t < n ? A[t + (int64_t)(n - 1) * lda] : 0.0;
  }
  __syncthreads();
  if (n == 1) {
    if (t == 0) d[0] = colbuf[0];
    return;
  }
  for (int q = n - 1; q >= 1; --q) {
    // ---- column q (in colbuf, updated up to the previous step): apply this
    // step's update (v, w; zero before the first), its diagonal to d[q], and
    // the reflector of entries 0..q-1 (alpha = entry q-1)
    const double wq = w[q], vq = v[q];
    double xr = 0.0;
    if (t <= q) xr = colbuf[t] - (v[t] * wq + w[t] * vq);
    if (t == q) d[q] = xr;
    double s2 = wave_sum_lane63(t < q - 1 ? xr * xr : 0.0);
    if (lane == 63) red[wv] = s2;
    if (t == q - 1) sc[2] = xr;
    __syncthreads();
    s2 = 0.0;
    for (int k = 0; k < kRgWaves; ++k) s2 += red[k];
    const double alpha = sc[2];
    double tau = 0.0, beta = alpha, scale = 1.0;
    if (s2 > 0.0) {
      const double nrm = sqrt(alpha * alpha + s2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    if (t < q - 1) {
      const double y = tau != 0.0 ? xr * scale : xr;
      A[t + (int64_t)q * lda] = y;
      vn[t] = y;
    } else if (t == q - 1) {
      A[t + (int64_t)q * lda] = beta;
      vn[t] = 1.0;
    } else if (t < kRgMaxN) {
      vn[t] = 0.0;
    }
    __syncthreads();
    // ---- sweep over the owned columns c < m = q: apply this step's update,
    // keep column m - 1 for the next step, accumulate p = A_new vn
    const int m = q;
    double vr[kRgChunks], wr[kRgChunks], vnr[kRgChunks], accr[kRgChunks];
#pragma unroll
    for (int k = 0; k < kRgChunks; ++k) {
      const int r = 64 * k + lane;
      vr[k] = r < m ? v[r] : 0.0;
      wr[k] = r < m ? w[r] : 0.0;
      vnr[k] = r < m ? vn[r] : 0.0;
      accr[k] = 0.0;
    }
#pragma unroll
    // columns in pairs (two independent reduction chains in flight); the
    // second column of a pair may lie beyond m, where v, w and vn read as
    // zero: its update subtracts zeros and it adds nothing to accr (its pc
    // entry is not read)
    for (int jp = 0; jp < kRgCols; jp += 2) {
      if (wv + kRgWaves * jp < m) {   // wave-uniform
        double col[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int j = jp + u;
          const int c = wv + kRgWaves * j;
          const double vc = v[c], wc = w[c], vnc = vn[c];
          col[u] = 0.0;
#pragma unroll
          for (int k = 0; k < rg_nch(j); ++k) {
            const int r = 64 * k + lane;
            const double x = a[rg_off(j) + k] - (vr[k] * wc + wr[k] * vc);
            if (k < rg_nch(j) - 1) {
              // rows of the earlier chunks all lie above the diagonal
              a[rg_off(j) + k] = x;
              col[u] += x * vnr[k];
              accr[k] += x * vnc;
            } else {
              // the last chunk holds the diagonal (vnr = vnc there)
              if (r <= c) {
                a[rg_off(j) + k] = x;
                col[u] += x * vnr[k];
              }
              if (r < c) accr[k] += x * vnc;
            }
            if (c == m - 1 && r <= c) colbuf[r] = x;
          }
        }
        const double s0 = wave_sum_lane63(col[0]);
        const double s1 = wave_sum_lane63(col[1]);
        if (lane == 63) {
          pc[wv + kRgWaves * jp] = s0;
          pc[wv + kRgWaves * (jp + 1)] = s1;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kRgChunks; ++k) part[(wv * kRgChunks + k) * 64 + lane] = accr[k];
    __syncthreads();
    // ---- p = A_new v' (thread t holds p_t), then
    //      w = tau p - (tau^2 / 2)(p . v') v' for the reflector just formed
    //      (v' = vn, length m), then v <- v'
    double pt = 0.0;
    if (t < m) {
      const int k = t >> 6, l = t & 63;
      pt = pc[t];
      for (int ww = 0; ww < kRgWaves; ++ww) pt += part[(ww * kRgChunks + k) * 64 + l];
    }
    if (t == 0) { e[q - 1] = beta; taus[q - 1] = tau; }
    const double wi = t < m ? tau * pt : 0.0;
    const double dotp = wave_sum_lane63(t < m ? wi * vn[t] : 0.0);
    if (lane == 63) red[wv] = dotp;
    __syncthreads();
    double dot = 0.0;
    for (int k = 0; k < kRgWaves; ++k) dot += red[k];
    if (t < kRgMaxN) {
      const double vt = t < m ? vn[t] : 0.0;
      w[t] = t < m ? wi - 0.5 * tau * dot * vt : 0.0;
      v[t] = vt;
    }
    __syncthreads();
  }
  // column 0: its diagonal after the last update
  if (t == 0) d[0] = colbuf[0] - 2.0 * v[0] * w[0];
}

// ---------------------------------------------------------------- Hermitian
// Complex (Bloch) blocks: the same one-workgroup reduction of a Hermitian
// matrix, H_i = I - tau v v^H with the complex tau of the standard Hermitian
// reduction, which makes the superdiagonal beta real (beta = -sign(Re alpha)
// |(alpha, x)|, tau = ((beta - Re alpha) / beta, -Im alpha / beta),
// v = x / (alpha - beta); tau = 0 when x = 0 and alpha is real):
//   p = A v,  w = tau p + alpha2 v,  alpha2 = -(tau / 2) (tau p)^H v,
//   A -= v w^H + w v^H.
// T is real (d, e); the reflectors stay in A's upper triangle as for real
// blocks, so the library's divide and conquer (complex eigenvector matrix)
// and back-transformation apply.
using zc = cplx<double>;

__device__ inline zc zc_div(zc a, zc b) {   // a / b (b != 0; scaled to avoid overflow)
  const double s = fabs(b.re) + fabs(b.im);
  const double br = b.re / s, bi = b.im / s;
  const double den = br * br + bi * bi;
  return {(a.re * br + a.im * bi) / (den * s), (a.im * br - a.re * bi) / (den * s)};
}

__device__ void hd_sweep(zc* __restrict__ A, int lda, int m, bool upd, const zc* v, const zc* w, const zc* vn,
                         zc* part, zc* p) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nrb = (m + 63) >> 6;
  const int g = kTdWaves / nrb;
  const int rb = wv % nrb, cg = wv / nrb;
  const int r = 64 * rb + lane;
  zc acc;
  if (cg < g && r < m) {
    const zc vr = v[r], wr = w[r];
    zc* col = A + r;
    int c = cg;
    for (; c + (kTdUnroll - 1) * g < m; c += kTdUnroll * g) {
      zc a[kTdUnroll];
#pragma unroll
      for (int u = 0; u < kTdUnroll; ++u) a[u] = col[(int64_t)(c + u * g) * lda];
#pragma unroll
      for (int u = 0; u < kTdUnroll; ++u) {
        const int cc = c + u * g;
        if (upd) {
          a[u] = a[u] - (vr * conj_(w[cc]) + wr * conj_(v[cc]));
          col[(int64_t)cc * lda] = a[u];
        }
        acc += a[u] * vn[cc];
      }
    }
    for (; c < m; c += g) {
      zc a = col[(int64_t)c * lda];
      if (upd) {
        a = a - (vr * conj_(w[c]) + wr * conj_(v[c]));
        col[(int64_t)c * lda] = a;
      }
      acc += a * vn[c];
    }
  }
  part[wv * 64 + lane] = acc;
  __syncthreads();
  if (threadIdx.x < m) {
    const int rr = threadIdx.x, b = rr >> 6, l = rr & 63;
    zc s;
    for (int k = 0; k < g; ++k) s += part[(k * nrb + b) * 64 + l];
    p[rr] = s;
  }
  __syncthreads();
}

// Reflector of column c from the values x_r (r < len) held by threads r
// (alpha = x_{len-1}); writes v (v[len-1] = 1), the scaled entries to
// A(0:len-2, c), beta to A(len-1, c); tau and beta through sc.
__device__ void hd_reflector(zc* __restrict__ A, int lda, int c, int len, zc xr, zc* vout, double* red,
                             double* sc) {
  const int t = threadIdx.x;
  const double s2 = td_block_sum(t < len - 1 ? abs2_(xr) : 0.0, red);
  if (t == len - 1) { sc[4] = xr.re; sc[5] = xr.im; }   // alpha
  __syncthreads();
  const zc alpha(sc[4], sc[5]);
  zc tau, scale(1.0, 0.0);
  double beta = alpha.re;
  if (s2 > 0.0 || alpha.im != 0.0) {
    const double nrm = sqrt(abs2_(alpha) + s2);
    beta = alpha.re >= 0.0 ? -nrm : nrm;
    tau = zc((beta - alpha.re) / beta, -alpha.im / beta);
    scale = zc_div(zc(1.0, 0.0), alpha - zc(beta, 0.0));
  }
  const bool refl = tau.re != 0.0 || tau.im != 0.0;
  if (t < len - 1) {
    const zc x = refl ? xr * scale : xr;
    A[t + (int64_t)c * lda] = x;
    vout[t] = x;
  } else if (t == len - 1) {
    A[t + (int64_t)c * lda] = zc(beta, 0.0);
    vout[t] = zc(1.0, 0.0);
  }
  if (t == 0) { sc[0] = tau.re; sc[1] = tau.im; sc[2] = beta; }
  __syncthreads();
}

__global__ __launch_bounds__(kTdThreads) void k_hetrd_small(zc* __restrict__ A, int n, int lda,
                                                            double* __restrict__ d, double* __restrict__ e,
                                                            zc* __restrict__ taus) {
  // (the complex type has constructors: LDS is declared as doubles)
  __shared__ __attribute__((aligned(16))) double lds_z[2 * (4 * kTdMaxN + kTdThreads)];
  zc* const v = reinterpret_cast<zc*>(lds_z);
  zc* const w = v + kTdMaxN;
  zc* const vn = w + kTdMaxN;
  zc* const p = vn + kTdMaxN;
  zc* const part = p + kTdMaxN;
  __shared__ double red[kTdWaves];
  __shared__ double sc[8];
  const int t = threadIdx.x;
  // the lower triangle from the upper one, conjugated
  for (int64_t q = t; q < (int64_t)n * n; q += kTdThreads) {
    const int r = (int)(q % n), c = (int)(q / n);
    if (r > c) A[r + (int64_t)c * lda] = conj_(A[c + (int64_t)r * lda]);
  }
  __syncthreads();
  if (t == 0) d[n - 1] = A[(n - 1) + (int64_t)(n - 1) * lda].re;
  if (n == 1) return;
  {
    const int len = n - 1;
    const zc x = t < len ? A[t + (int64_t)(n - 1) * lda] : zc();
    hd_reflector(A, lda, n - 1, len, x, v, red, sc);
    hd_sweep(A, lda, len, false, v, v, v, part, p);
  }
  for (int i = n - 2; i >= 0; --i) {
    // v, p = A(0:i,0:i) v and tau of step i are ready
    const zc tau(sc[0], sc[1]);
    const double beta = sc[2];
    const zc wi = t <= i ? tau * p[t] : zc();
    const zc pr = t <= i ? conj_(wi) * v[t] : zc();   // (tau p)^H v, term t
    const double dre = td_block_sum(pr.re, red);
    const double dim = td_block_sum(pr.im, red);
    const zc a2 = (-0.5) * (tau * zc(dre, dim));
    if (t <= i) w[t] = wi + a2 * v[t];
    if (t == 0) { e[i] = beta; taus[i] = tau; }
    __syncthreads();
    const bool refl = tau.re != 0.0 || tau.im != 0.0;
    if (i == 0) {
      if (t == 0) d[0] = A[0].re - (refl ? 2.0 * (v[0] * conj_(w[0])).re : 0.0);
      break;
    }
    // column i of the updated block (entries r < i) and its diagonal
    zc xr;
    if (t < i) {
      xr = A[t + (int64_t)i * lda];
      if (refl) xr = xr - (v[t] * conj_(w[i]) + w[t] * conj_(v[i]));
    }
    if (t == i) d[i] = A[i + (int64_t)i * lda].re - (refl ? 2.0 * (v[i] * conj_(w[i])).re : 0.0);
    hd_reflector(A, lda, i, i, xr, vn, red, sc);
    hd_sweep(A, lda, i, refl, v, w, vn, part, p);
    if (t < i) v[t] = vn[t];
    __syncthreads();
  }
}

}  // namespace

bool hetrd_small_ok(int n) { return n >= 1 && n <= kTdMaxN; }

void launch_hetrd_small(cplx<double>* A, int n, int lda, double* d, double* e, cplx<double>* tau, hipStream_t st) {
  launch_k(k_hetrd_small, 1, kTdThreads, 0, st, A, n, lda, d, e, tau);
}

bool sytrd_small_ok(int n) { return n >= 1 && n <= kTdMaxN; }

void launch_sytrd_small(double* A, int n, int lda, double* d, double* e, double* tau, hipStream_t st) {
  if (n <= kRgMaxN)
    launch_k(k_sytrd_reg, 1, kRgThreads, 0, st, A, n, lda, d, e, tau);
  else
    launch_k(k_sytrd_small, 1, kTdThreads, 0, st, A, n, lda, d, e, tau);
}

}  // namespace hcu
