// Learned initial guess of the Hubbard occupation matrices (the paper starts
// from the isolated-atom average occupation, Sec. II.B; this replaces that
// start by a prediction from the local environment):
//
//   site descriptor  G[32 S + k] = sum_{J in species S, images}
//                        exp(-(r - mu_k)^2 / (2 w^2)) (cos(pi r / rc) + 1) / 2,
//                    mu_k = 1 + 5.5 k / 31, w = 0.25, rc = 6.5 (bohr);
//   site frame       flag 1 when the apical O neighbours (r < 4.5, |dz| < 1)
//                    lie along (1, -1, 0): the rutile sublattice rotated by
//                    90 degrees about z;
//   MLP              dims[0] -> ... -> dims[L], SiLU between layers, linear
//                    output, standardised inputs and outputs;
//   guess            15 local-frame entries of D -> rotate back, symmetrise,
//                    clip the spectrum to [0, 1].
//
// Training (FP32) and inference (FP32 or BF16 operands with FP32
// accumulation) run on the matrix cores through one small GEMM kernel per
// precision with fused bias / SiLU / SiLU-derivative epilogues.
#include "common.h"

#include <cmath>
#include <cstring>
#include <string>

namespace hcu {

constexpr int kNG = 32;
constexpr double kMuLo = 1.0, kMuHi = 6.5, kGw = 0.25, kRc = 6.5;
constexpr int kNShell = 15;
constexpr double kShellLo = 0.5, kShellHi = 4.0;
constexpr double kApicalR = 4.5, kApicalDz = 1.0;

__device__ inline float silu_f(float z) { return z / (1.0f + expf(-z)); }
__device__ inline float silu_grad_f(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// bf16 <-> f32 (round to nearest even; finite inputs)
__device__ inline unsigned short to_bf16(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// ---------------------------------------------------------------- GEMM (FP32)
// C(i, j) = sum_k A(i, k) B(k, j), A(i, k) = A[i sai + k sak],
// B(k, j) = B[k sbk + j sbj]; one wave per 16 x 16 tile.
// mode 0: C = acc;  mode 1: Z = acc + bias[j], H = silu(Z) if H != null;
// mode 2: C = acc * silu'(Zp).
__global__ __launch_bounds__(64) void k_gemm_f32(int M, int N, int K, const float* __restrict__ A, int64_t sai,
                                                 int64_t sak, const float* __restrict__ B, int64_t sbk, int64_t sbj,
                                                 float* __restrict__ C, int64_t ldc, const float* __restrict__ bias,
                                                 float* __restrict__ H, const float* __restrict__ Zp, int mode) {
  const int lane = threadIdx.x;
  const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
  const int ia = i0 + (lane & 15), jb = j0 + (lane & 15);
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int k = k0 + (lane >> 4);
    const float a = (ia < M && k < K) ? A[(int64_t)ia * sai + (int64_t)k * sak] : 0.f;
    const float b = (jb < N && k < K) ? B[(int64_t)k * sbk + (int64_t)jb * sbj] : 0.f;
    acc = Mf<float>::mfma(a, b, acc);
  }
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + Mf<float>::row(lane, r);
    const int j = jb;
    if (i >= M || j >= N) continue;
    const int64_t o = (int64_t)i * ldc + j;
    if (mode == 0) {
      C[o] = acc[r];
    } else if (mode == 1) {
      const float z = acc[r] + bias[j];
      C[o] = z;
      if (H) H[o] = silu_f(z);
    } else {
      C[o] = acc[r] * silu_grad_f(Zp[o]);
    }
  }
}

// ---------------------------------------------------------------- GEMM (BF16)
// Z = A W^T + bias with A [M x K] and W [N x K] in bf16, FP32 accumulation;
// out: bf16 silu(Z) (hidden layers) or FP32 Z (last layer).
typedef short s4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(64) void k_gemm_bf16(int M, int N, int K, const unsigned short* __restrict__ A,
                                                  const unsigned short* __restrict__ W,
                                                  const float* __restrict__ bias, unsigned short* __restrict__ Hb,
                                                  float* __restrict__ Y) {
  const int lane = threadIdx.x;
  const int i0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
  const int ia = i0 + (lane & 15), jb = j0 + (lane & 15);
  f4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    const int kb = k0 + 4 * (lane >> 4);
    s4 a, b;
    for (int v = 0; v < 4; ++v) {
      a[v] = (ia < M && kb + v < K) ? (short)A[(int64_t)ia * K + kb + v] : (short)0;
      b[v] = (jb < N && kb + v < K) ? (short)W[(int64_t)jb * K + kb + v] : (short)0;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + Mf<float>::row(lane, r);
    if (i >= M || jb >= N) continue;
    const float z = acc[r] + bias[jb];
    if (Hb) Hb[(int64_t)i * N + jb] = to_bf16(silu_f(z));
    else Y[(int64_t)i * N + jb] = z;
  }
}

__global__ void k_to_bf16(const float* __restrict__ x, unsigned short* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = to_bf16(x[i]);
}

// H0 = (X[idx] - mean) / std, FP32 or bf16 output
__global__ void k_standardise(const float* __restrict__ X, const int* __restrict__ idx, int rows, int cols,
                              const float* __restrict__ mean, const float* __restrict__ sd, float* __restrict__ H,
                              unsigned short* __restrict__ Hb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)rows * cols) return;
  const int b = (int)(e / cols), k = (int)(e % cols);
  const int src = idx ? idx[b] : b;
  const float v = (X[(int64_t)src * cols + k] - mean[k]) / sd[k];
  if (H) H[e] = v;
  if (Hb) Hb[e] = to_bf16(v);
}

__global__ void k_destandardise(float* __restrict__ Y, int rows, int cols, const float* __restrict__ mean,
                                const float* __restrict__ sd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)rows * cols) return;
  const int k = (int)(e % cols);
  Y[e] = Y[e] * sd[k] + mean[k];
}

// column mean and standard deviation (two passes, FP64 sums); a deviation
// below 1e-6 is replaced by 1 (constant columns)
__global__ void k_colstats(const float* __restrict__ X, int rows, int cols, float* __restrict__ mean,
                           float* __restrict__ sd) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= cols) return;
  double s = 0;
  for (int r = 0; r < rows; ++r) s += X[(int64_t)r * cols + k];
  const double m = rows > 0 ? s / rows : 0.0;
  double v = 0;
  for (int r = 0; r < rows; ++r) {
    const double d = X[(int64_t)r * cols + k] - m;
    v += d * d;
  }
  const double sdev = rows > 0 ? sqrt(v / rows) : 1.0;
  mean[k] = (float)m;
  sd[k] = sdev > 1e-6 ? (float)sdev : 1.0f;
}

// MSE against standardised targets: dY = 2 (Y - t) / (B n); block partial
// sums of (Y - t)^2 in part[blockIdx.x] (fixed grid, fixed tree).
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ Y, const float* __restrict__ T,
                                             const int* __restrict__ idx, int rows, int cols,
                                             const float* __restrict__ mean, const float* __restrict__ sd,
                                             float* __restrict__ dY, double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t n = (int64_t)rows * cols;
  const float scale = 2.0f / (float)n;
  double acc = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / cols), k = (int)(e % cols);
    const int src = idx ? idx[b] : b;
    const float t = (T[(int64_t)src * cols + k] - mean[k]) / sd[k];
    const float d = Y[e] - t;
    dY[e] = scale * d;
    acc += (double)d * d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// db[j] = sum_b G[b][j]: one workgroup per column, fixed tree
__global__ __launch_bounds__(256) void k_colsum(const float* __restrict__ G, int rows, int cols,
                                                float* __restrict__ db) {
  __shared__ float red[256];
  const int j = blockIdx.x;
  float acc = 0.f;
  for (int r = threadIdx.x; r < rows; r += blockDim.x) acc += G[(int64_t)r * cols + j];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[j] = red[0];
}

__global__ void k_adam(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ Mm,
                       float* __restrict__ Vv, int64_t n, float lr, float b1, float b2, float eps, float bc1,
                       float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = G[i];
  const float m = b1 * Mm[i] + (1.0f - b1) * g;
  const float v = b2 * Vv[i] + (1.0f - b2) * g * g;
  Mm[i] = m;
  Vv[i] = v;
  P[i] -= lr * (m / bc1) / (sqrtf(v / bc2) + eps);
}

// ---------------------------------------------------------------- descriptor
// One workgroup per Hubbard site; thread t < 32 nspecies computes entry t by
// a fixed-order sum over atoms and images; thread 0 also sums the apical
// dx*dy for the frame flag.
__global__ void k_descriptor(int nhub, const int* __restrict__ hub_atom, int natom, const double* __restrict__ pos,
                             const int* __restrict__ spec, const int* __restrict__ spec_hub, int nspecies, double L0,
                             double L1, double L2, int ni0, int ni1, int ni2, float* __restrict__ desc,
                             int* __restrict__ flags) {
  const int site = blockIdx.x;
  const int t = threadIdx.x;
  const int ia = hub_atom[site];
  const double xi = pos[3 * ia], yi = pos[3 * ia + 1], zi = pos[3 * ia + 2];
  const int nout = kNG * nspecies;
  if (t < nout) {
    const int S = t / kNG, k = t % kNG;
    const double mu = kMuLo + (kMuHi - kMuLo) * k / (kNG - 1);
    double acc = 0;
    for (int j = 0; j < natom; ++j) {
      if (spec[j] != S) continue;
      for (int a = -ni0; a <= ni0; ++a)
        for (int b = -ni1; b <= ni1; ++b)
          for (int c = -ni2; c <= ni2; ++c) {
            const double dx = pos[3 * j] + a * L0 - xi, dy = pos[3 * j + 1] + b * L1 - yi,
                         dz = pos[3 * j + 2] + c * L2 - zi;
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r > 0 && r < kRc) {
              const double u = (r - mu) / kGw;
              acc += exp(-0.5 * u * u) * 0.5 * (cos(M_PI * r / kRc) + 1.0);
            }
          }
    }
    desc[(int64_t)site * nout + t] = (float)acc;
  }
  if (t == 0) {
    double ap = 0;
    for (int j = 0; j < natom; ++j) {
      if (spec_hub[spec[j]]) continue;
      for (int a = -ni0; a <= ni0; ++a)
        for (int b = -ni1; b <= ni1; ++b)
          for (int c = -ni2; c <= ni2; ++c) {
            const double dx = pos[3 * j] + a * L0 - xi, dy = pos[3 * j + 1] + b * L1 - yi,
                         dz = pos[3 * j + 2] + c * L2 - zi;
            const double r = sqrt(dx * dx + dy * dy + dz * dz);
            if (r > 0 && r < kApicalR && fabs(dz) < kApicalDz) ap += dx * dy;
          }
    }
    flags[site] = ap < 0 ? 1 : 0;
  }
}

// ---------------------------------------------------------------- density shells
// part[site][chunk][0..14] = sum_x rho(x) g_k(x), [15..29] = sum_x g_k(x),
// g_k(x) = sum_T exp(-(|x - R - T| - r_k)^2 / (2 w^2)), rho summed over spins.
__global__ __launch_bounds__(256) void k_shells(const double* __restrict__ rho, int nspin, int nd, int n1, int n2,
                                                double h0, double h1, double h2, double L0, double L1, double L2,
                                                int ni0, int ni1, int ni2, const double* __restrict__ sites,
                                                int nchunks, double* __restrict__ part) {
  __shared__ double red[256];
  const int site = blockIdx.y, chunk = blockIdx.x;
  const double X = sites[3 * site], Yc = sites[3 * site + 1], Zc = sites[3 * site + 2];
  const int per = (nd + nchunks - 1) / nchunks;
  const int p0 = chunk * per, p1 = min(nd, p0 + per);
  double num[kNShell], den[kNShell];
  for (int k = 0; k < kNShell; ++k) num[k] = den[k] = 0;
  for (int p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    const int i = p % n1, j = (p / n1) % n2, l = p / (n1 * n2);
    double rv = 0;
    for (int s = 0; s < nspin; ++s) rv += rho[(int64_t)s * nd + p];
    for (int a = -ni0; a <= ni0; ++a)
      for (int b = -ni1; b <= ni1; ++b)
        for (int c = -ni2; c <= ni2; ++c) {
          const double dx = i * h0 - X - a * L0, dy = j * h1 - Yc - b * L1, dz = l * h2 - Zc - c * L2;
          const double r = sqrt(dx * dx + dy * dy + dz * dz);
          for (int k = 0; k < kNShell; ++k) {
            const double u = (r - (kShellLo + (kShellHi - kShellLo) * k / (kNShell - 1))) / kGw;
            const double g = exp(-0.5 * u * u);
            num[k] += g * rv;
            den[k] += g;
          }
        }
  }
  for (int q = 0; q < 2 * kNShell; ++q) {
    red[threadIdx.x] = q < kNShell ? num[q] : den[q - kNShell];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[((int64_t)site * nchunks + chunk) * 2 * kNShell + q] = red[0];
    __syncthreads();
  }
}

}  // namespace hcu

using namespace hcu;

// ====================================================================== MLP object
struct hcu_mlp {
  std::vector<int> dims;
  int nl = 0;
  int max_batch = 0;
  int64_t np = 0;
  std::vector<int64_t> woff, bo;   // per-layer weight / bias offsets in the flat parameter vector
  int maxw = 0;
  hipStream_t stream = nullptr;
  bool bound = false;
  bool scaled = false;
  bool bf16_dirty = true;
  int step = 0;
  std::string err;
  // device
  float *P = nullptr, *G = nullptr, *Mm = nullptr, *Vv = nullptr;
  unsigned short* Pb = nullptr;
  float *in_mean = nullptr, *in_sd = nullptr, *out_mean = nullptr, *out_sd = nullptr;
  std::vector<float*> H, Z;      // H[0..nl], Z[0..nl-1]
  float *gA = nullptr, *gB = nullptr;
  unsigned short *hb0 = nullptr, *hb1 = nullptr;
  float* Xin = nullptr;          // descriptor staging for hcu_mlp_guess
  double* part = nullptr;
};

namespace {
constexpr int kMsePart = 256;

hcu_status mfail(hcu_mlp* m, hcu_status s, const std::string& msg) {
  m->err = msg;
  return s;
}

#define MLP_HIP(m, call)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) return mfail((m), HCU_DEVICE, std::string("HIP: ") + hipGetErrorString(e_)); \
  } while (0)

size_t mlp_layout(hcu_mlp& m, char* base) {
  size_t off = 0;
  auto take = [&](auto*& ptr, size_t bytes) {
    off = (off + 255) & ~size_t(255);
    ptr = base ? reinterpret_cast<std::remove_reference_t<decltype(ptr)>>(base + off) : nullptr;
    off += std::max<size_t>(bytes, 1);
  };
  const size_t nb = (size_t)m.max_batch;
  take(m.P, 4 * m.np);
  take(m.G, 4 * m.np);
  take(m.Mm, 4 * m.np);
  take(m.Vv, 4 * m.np);
  take(m.Pb, 2 * m.np);
  take(m.in_mean, 4 * m.dims[0]);
  take(m.in_sd, 4 * m.dims[0]);
  take(m.out_mean, 4 * m.dims[m.nl]);
  take(m.out_sd, 4 * m.dims[m.nl]);
  m.H.assign(m.nl + 1, nullptr);
  m.Z.assign(m.nl, nullptr);
  for (int l = 0; l <= m.nl; ++l) take(m.H[l], 4 * nb * m.dims[l]);
  for (int l = 0; l < m.nl; ++l) take(m.Z[l], 4 * nb * m.dims[l + 1]);
  take(m.gA, 4 * nb * m.maxw);
  take(m.gB, 4 * nb * m.maxw);
  take(m.hb0, 2 * nb * m.maxw);
  take(m.hb1, 2 * nb * m.maxw);
  take(m.Xin, 4 * nb * m.dims[0]);
  take(m.part, sizeof(double) * kMsePart);
  return off;
}

hcu_status mlp_check(hcu_mlp* m, int batch) {
  if (!m) return HCU_INVALID_ARG;
  if (!m->bound) return mfail(m, HCU_NOT_BOUND, "MLP not bound to a workspace");
  if (!m->scaled) return mfail(m, HCU_INVALID_ARG, "MLP scaling not set");
  if (batch < 1 || batch > m->max_batch) return mfail(m, HCU_INVALID_ARG, "batch outside 1..max_batch");
  return HCU_OK;
}

void gemm_f32(hcu_mlp& m, int M, int N, int K, const float* A, int64_t sai, int64_t sak, const float* B, int64_t sbk,
              int64_t sbj, float* C, int64_t ldc, const float* bias, float* H, const float* Zp, int mode) {
  dim3 grid((M + 15) / 16, (N + 15) / 16);
  k_gemm_f32<<<grid, 64, 0, m.stream>>>(M, N, K, A, sai, sak, B, sbk, sbj, C, ldc, bias, H, Zp, mode);
}

// FP32 forward of rows X[idx] (raw): H[0] standardised, Z[l], H[l+1];
// H[nl] = standardised output.
void forward_f32(hcu_mlp& m, const float* X, const int* idx, int B) {
  const int64_t n0 = (int64_t)B * m.dims[0];
  k_standardise<<<(unsigned)((n0 + 255) / 256), 256, 0, m.stream>>>(X, idx, B, m.dims[0], m.in_mean, m.in_sd, m.H[0],
                                                                    nullptr);
  for (int l = 0; l < m.nl; ++l) {
    const int K = m.dims[l], N = m.dims[l + 1];
    const bool last = l == m.nl - 1;
    gemm_f32(m, B, N, K, m.H[l], K, 1, m.P + m.woff[l], 1, K, last ? m.H[l + 1] : m.Z[l], N, m.P + m.bo[l],
             last ? nullptr : m.H[l + 1], nullptr, 1);
  }
}

hcu_status loss_and_grad(hcu_mlp& m, const float* X, const float* T, const int* idx, int B, double* loss) {
  forward_f32(m, X, idx, B);
  const int no = m.dims[m.nl];
  k_mse<<<kMsePart, 256, 0, m.stream>>>(m.H[m.nl], T, idx, B, no, m.out_mean, m.out_sd, m.gA, m.part);
  float* g = m.gA;
  float* gn = m.gB;
  for (int l = m.nl - 1; l >= 0; --l) {
    const int K = m.dims[l], N = m.dims[l + 1];
    // dW[N x K] = g^T H[l]
    gemm_f32(m, N, K, B, g, 1, N, m.H[l], K, 1, m.G + m.woff[l], K, nullptr, nullptr, nullptr, 0);
    k_colsum<<<N, 256, 0, m.stream>>>(g, B, N, m.G + m.bo[l]);
    if (l > 0) {
      // g_prev[B x K] = (g W) * silu'(Z[l-1])
      gemm_f32(m, B, K, N, g, N, 1, m.P + m.woff[l], K, 1, gn, K, nullptr, nullptr, m.Z[l - 1], 2);
      std::swap(g, gn);
    }
  }
  MLP_HIP(&m, hipGetLastError());
  if (loss) {
    double hp[kMsePart];
    MLP_HIP(&m, hipMemcpyAsync(hp, m.part, sizeof(hp), hipMemcpyDeviceToHost, m.stream));
    MLP_HIP(&m, hipStreamSynchronize(m.stream));
    double s = 0;
    for (int i = 0; i < kMsePart; ++i) s += hp[i];
    *loss = s / ((double)B * no);
  }
  return HCU_OK;
}

// Forward to physical outputs Y [B x n_out] (device, FP32).
hcu_status forward_out(hcu_mlp& m, const float* X, int B, float* Y, int bf16) {
  const int no = m.dims[m.nl];
  if (!bf16) {
    forward_f32(m, X, nullptr, B);
    MLP_HIP(&m, hipMemcpyAsync(Y, m.H[m.nl], sizeof(float) * B * no, hipMemcpyDeviceToDevice, m.stream));
  } else {
    if (m.bf16_dirty) {
      k_to_bf16<<<(unsigned)((m.np + 255) / 256), 256, 0, m.stream>>>(m.P, m.Pb, m.np);
      m.bf16_dirty = false;
    }
    const int64_t n0 = (int64_t)B * m.dims[0];
    k_standardise<<<(unsigned)((n0 + 255) / 256), 256, 0, m.stream>>>(X, nullptr, B, m.dims[0], m.in_mean, m.in_sd,
                                                                      nullptr, m.hb0);
    unsigned short* a = m.hb0;
    unsigned short* b = m.hb1;
    for (int l = 0; l < m.nl; ++l) {
      const int K = m.dims[l], N = m.dims[l + 1];
      const bool last = l == m.nl - 1;
      dim3 grid((B + 15) / 16, (N + 15) / 16);
      k_gemm_bf16<<<grid, 64, 0, m.stream>>>(B, N, K, a, m.Pb + m.woff[l], m.P + m.bo[l], last ? nullptr : b,
                                             last ? Y : nullptr);
      std::swap(a, b);
    }
  }
  const int64_t ny = (int64_t)B * no;
  k_destandardise<<<(unsigned)((ny + 255) / 256), 256, 0, m.stream>>>(Y, B, no, m.out_mean, m.out_sd);
  MLP_HIP(&m, hipGetLastError());
  return HCU_OK;
}

// 5 x 5 symmetric eigen-decomposition by cyclic Jacobi (host, FP64)
void jacobi5(double A[5][5], double w[5], double V[5][5]) {
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) V[i][j] = i == j;
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = 0;
    for (int i = 0; i < 5; ++i)
      for (int j = i + 1; j < 5; ++j) off += A[i][j] * A[i][j];
    if (off < 1e-30) break;
    for (int p = 0; p < 5; ++p)
      for (int q = p + 1; q < 5; ++q) {
        if (std::fabs(A[p][q]) < 1e-300) continue;
        const double th = (A[q][q] - A[p][p]) / (2 * A[p][q]);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1));
        const double c = 1 / std::sqrt(t * t + 1), s = t * c;
        for (int k = 0; k < 5; ++k) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 5; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 5; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < 5; ++i) w[i] = A[i][i];
}

// the signed permutation of the real d orbitals (xy, yz, z^2, xz, x^2-y^2)
// under (x, y, z) -> (y, -x, z)
constexpr double kFrame[5][5] = {{-1, 0, 0, 0, 0}, {0, 0, 0, -1, 0}, {0, 0, 1, 0, 0}, {0, 1, 0, 0, 0}, {0, 0, 0, 0, -1}};

void occupation_from_output(const float* y15, int flag, double D[5][5]) {
  double Dl[5][5];
  int t = 0;
  for (int i = 0; i < 5; ++i)
    for (int j = i; j < 5; ++j) {
      Dl[i][j] = Dl[j][i] = y15[t];
      ++t;
    }
  double R[5][5];
  if (flag) {   // D = M^T Dl M
    double T1[5][5];
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) {
        double s = 0;
        for (int k = 0; k < 5; ++k) s += Dl[i][k] * kFrame[k][j];
        T1[i][j] = s;
      }
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) {
        double s = 0;
        for (int k = 0; k < 5; ++k) s += kFrame[k][i] * T1[k][j];
        R[i][j] = s;
      }
  } else {
    std::memcpy(R, Dl, sizeof(R));
  }
  for (int i = 0; i < 5; ++i)
    for (int j = i + 1; j < 5; ++j) R[i][j] = R[j][i] = 0.5 * (R[i][j] + R[j][i]);
  double w[5], V[5][5];
  jacobi5(R, w, V);
  for (int i = 0; i < 5; ++i) w[i] = std::min(1.0, std::max(0.0, w[i]));
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) {
      double s = 0;
      for (int k = 0; k < 5; ++k) s += V[i][k] * w[k] * V[j][k];
      D[i][j] = s;
    }
}

void image_counts(const Ctx& c, double reach, int ni[3]) {
  for (int a = 0; a < 3; ++a) ni[a] = (int)std::ceil(reach / c.p.L[a]);
}

// Descriptors of the context's Hubbard sites into desc (device) and their
// frame flags into flags_host.
hcu_status run_descriptor(Ctx& c, float* desc, int* flags_host) {
  const int nh = (int)c.hub_atoms.size();
  const int na = c.p.natom;
  const int nsp = c.p.nspecies;
  // scratch in d_red: pos (3 na doubles), species (na ints), hub atoms, species flags, frame flags
  char* base = reinterpret_cast<char*>(c.d_red);
  double* d_pos = reinterpret_cast<double*>(base);
  int* d_spec = reinterpret_cast<int*>(base + sizeof(double) * 3 * na);
  int* d_hub = d_spec + na;
  int* d_sh = d_hub + nh;
  int* d_flags = d_sh + nsp;
  std::vector<int> sh(nsp);
  for (int s = 0; s < nsp; ++s) sh[s] = c.species[s].hub_l >= 0 ? 1 : 0;
  HCU_HIP(hipMemcpyAsync(d_pos, c.pos.data(), sizeof(double) * 3 * na, hipMemcpyHostToDevice, c.stream));
  HCU_HIP(hipMemcpyAsync(d_spec, c.atom_species.data(), sizeof(int) * na, hipMemcpyHostToDevice, c.stream));
  HCU_HIP(hipMemcpyAsync(d_hub, c.hub_atoms.data(), sizeof(int) * nh, hipMemcpyHostToDevice, c.stream));
  HCU_HIP(hipMemcpyAsync(d_sh, sh.data(), sizeof(int) * nsp, hipMemcpyHostToDevice, c.stream));
  int ni[3];
  image_counts(c, kRc, ni);
  const int threads = std::max(64, (kNG * nsp + 63) / 64 * 64);
  k_descriptor<<<nh, threads, 0, c.stream>>>(nh, d_hub, na, d_pos, d_spec, d_sh, nsp, c.p.L[0], c.p.L[1], c.p.L[2],
                                             ni[0], ni[1], ni[2], desc, d_flags);
  HCU_HIP(hipGetLastError());
  HCU_HIP(hipMemcpyAsync(flags_host, d_flags, sizeof(int) * nh, hipMemcpyDeviceToHost, c.stream));
  HCU_HIP(hipStreamSynchronize(c.stream));
  return HCU_OK;
}

size_t descriptor_scratch_bytes(const Ctx& c) {
  return sizeof(double) * 3 * c.p.natom + sizeof(int) * (c.p.natom + 2 * c.hub_atoms.size() + c.p.nspecies);
}
}  // namespace

extern "C" {

hcu_status hcu_mlp_create(const int* dims, int nlayers, int max_batch, hcu_mlp** out) {
  if (!dims || !out || nlayers < 1 || nlayers > 8 || max_batch < 1) return HCU_INVALID_ARG;
  *out = nullptr;
  hcu_mlp* m = new (std::nothrow) hcu_mlp();
  if (!m) return HCU_OOM;
  *out = m;
  m->nl = nlayers;
  m->max_batch = max_batch;
  m->dims.assign(dims, dims + nlayers + 1);
  for (int d : m->dims)
    if (d < 1 || d > 4096) return mfail(m, HCU_INVALID_ARG, "layer widths must be in 1..4096");
  int64_t o = 0;
  for (int l = 0; l < nlayers; ++l) {
    m->woff.push_back(o);
    o += (int64_t)m->dims[l] * m->dims[l + 1];
    m->bo.push_back(o);
    o += m->dims[l + 1];
  }
  m->np = o;
  m->maxw = *std::max_element(m->dims.begin(), m->dims.end());
  return HCU_OK;
}

void hcu_mlp_destroy(hcu_mlp* m) { delete m; }

const char* hcu_mlp_last_error(const hcu_mlp* m) { return m ? m->err.c_str() : "null MLP"; }

hcu_status hcu_mlp_param_count(const hcu_mlp* m, int64_t* n) {
  if (!m || !n) return HCU_INVALID_ARG;
  *n = m->np;
  return HCU_OK;
}

hcu_status hcu_mlp_workspace_size(hcu_mlp* m, size_t* bytes) {
  if (!m || !bytes) return HCU_INVALID_ARG;
  *bytes = mlp_layout(*m, nullptr);
  return HCU_OK;
}

hcu_status hcu_mlp_bind(hcu_mlp* m, void* dev, size_t bytes, void* stream) {
  if (!m || !dev) return HCU_INVALID_ARG;
  if (reinterpret_cast<uintptr_t>(dev) % 256 != 0) return mfail(m, HCU_INVALID_ARG, "workspace must be 256-byte aligned");
  if (bytes < mlp_layout(*m, nullptr)) return mfail(m, HCU_INVALID_ARG, "workspace too small");
  mlp_layout(*m, reinterpret_cast<char*>(dev));
  m->stream = reinterpret_cast<hipStream_t>(stream);
  MLP_HIP(m, hipMemsetAsync(m->Mm, 0, 4 * m->np, m->stream));
  MLP_HIP(m, hipMemsetAsync(m->Vv, 0, 4 * m->np, m->stream));
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  m->bound = true;
  m->step = 0;
  return HCU_OK;
}

hcu_status hcu_mlp_set_params(hcu_mlp* m, const float* p) {
  if (!m || !p) return HCU_INVALID_ARG;
  if (!m->bound) return mfail(m, HCU_NOT_BOUND, "MLP not bound");
  for (int64_t i = 0; i < m->np; ++i)
    if (!std::isfinite(p[i])) return mfail(m, HCU_NAN, "non-finite parameter");
  MLP_HIP(m, hipMemcpyAsync(m->P, p, 4 * m->np, hipMemcpyHostToDevice, m->stream));
  MLP_HIP(m, hipMemsetAsync(m->Mm, 0, 4 * m->np, m->stream));
  MLP_HIP(m, hipMemsetAsync(m->Vv, 0, 4 * m->np, m->stream));
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  m->step = 0;
  m->bf16_dirty = true;
  return HCU_OK;
}

hcu_status hcu_mlp_get_params(hcu_mlp* m, float* p) {
  if (!m || !p) return HCU_INVALID_ARG;
  if (!m->bound) return mfail(m, HCU_NOT_BOUND, "MLP not bound");
  MLP_HIP(m, hipMemcpyAsync(p, m->P, 4 * m->np, hipMemcpyDeviceToHost, m->stream));
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  return HCU_OK;
}

hcu_status hcu_mlp_set_scaling(hcu_mlp* m, const float* in_mean, const float* in_sd, const float* out_mean,
                               const float* out_sd) {
  if (!m || !in_mean || !in_sd || !out_mean || !out_sd) return HCU_INVALID_ARG;
  if (!m->bound) return mfail(m, HCU_NOT_BOUND, "MLP not bound");
  const int d0 = m->dims[0], dl = m->dims[m->nl];
  for (int i = 0; i < d0; ++i)
    if (!(in_sd[i] > 0)) return mfail(m, HCU_INVALID_ARG, "input deviations must be positive");
  for (int i = 0; i < dl; ++i)
    if (!(out_sd[i] > 0)) return mfail(m, HCU_INVALID_ARG, "output deviations must be positive");
  MLP_HIP(m, hipMemcpyAsync(m->in_mean, in_mean, 4 * d0, hipMemcpyHostToDevice, m->stream));
  MLP_HIP(m, hipMemcpyAsync(m->in_sd, in_sd, 4 * d0, hipMemcpyHostToDevice, m->stream));
  MLP_HIP(m, hipMemcpyAsync(m->out_mean, out_mean, 4 * dl, hipMemcpyHostToDevice, m->stream));
  MLP_HIP(m, hipMemcpyAsync(m->out_sd, out_sd, 4 * dl, hipMemcpyHostToDevice, m->stream));
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  m->scaled = true;
  return HCU_OK;
}

hcu_status hcu_mlp_fit_scaling(hcu_mlp* m, const float* X, const float* T, int rows) {
  if (!m || !X || !T || rows < 1) return HCU_INVALID_ARG;
  if (!m->bound) return mfail(m, HCU_NOT_BOUND, "MLP not bound");
  const int d0 = m->dims[0], dl = m->dims[m->nl];
  k_colstats<<<(d0 + 63) / 64, 64, 0, m->stream>>>(X, rows, d0, m->in_mean, m->in_sd);
  k_colstats<<<(dl + 63) / 64, 64, 0, m->stream>>>(T, rows, dl, m->out_mean, m->out_sd);
  MLP_HIP(m, hipGetLastError());
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  m->scaled = true;
  return HCU_OK;
}

hcu_status hcu_mlp_get_scaling(hcu_mlp* m, float* in_mean, float* in_sd, float* out_mean, float* out_sd) {
  if (!m || !in_mean || !in_sd || !out_mean || !out_sd) return HCU_INVALID_ARG;
  if (!m->bound || !m->scaled) return mfail(m, HCU_INVALID_ARG, "MLP scaling not set");
  const int d0 = m->dims[0], dl = m->dims[m->nl];
  MLP_HIP(m, hipMemcpyAsync(in_mean, m->in_mean, 4 * d0, hipMemcpyDeviceToHost, m->stream));
  MLP_HIP(m, hipMemcpyAsync(in_sd, m->in_sd, 4 * d0, hipMemcpyDeviceToHost, m->stream));
  MLP_HIP(m, hipMemcpyAsync(out_mean, m->out_mean, 4 * dl, hipMemcpyDeviceToHost, m->stream));
  MLP_HIP(m, hipMemcpyAsync(out_sd, m->out_sd, 4 * dl, hipMemcpyDeviceToHost, m->stream));
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  return HCU_OK;
}

hcu_status hcu_mlp_forward(hcu_mlp* m, const float* X, int batch, float* Y, int bf16) {
  hcu_status s = mlp_check(m, batch);
  if (s != HCU_OK) return s;
  if (!X || !Y) return mfail(m, HCU_INVALID_ARG, "null input/output");
  s = forward_out(*m, X, batch, Y, bf16);
  if (s != HCU_OK) return s;
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  return HCU_OK;
}

hcu_status hcu_mlp_gradient(hcu_mlp* m, const float* X, const float* T, const int* idx, int batch, float* grad,
                            double* loss) {
  hcu_status s = mlp_check(m, batch);
  if (s != HCU_OK) return s;
  if (!X || !T || !grad || !loss) return mfail(m, HCU_INVALID_ARG, "null argument");
  s = loss_and_grad(*m, X, T, idx, batch, loss);
  if (s != HCU_OK) return s;
  MLP_HIP(m, hipMemcpyAsync(grad, m->G, 4 * m->np, hipMemcpyDeviceToHost, m->stream));
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  return HCU_OK;
}

hcu_status hcu_mlp_train_step(hcu_mlp* m, const float* X, const float* T, const int* idx, int batch, float lr,
                              double* loss) {
  hcu_status s = mlp_check(m, batch);
  if (s != HCU_OK) return s;
  if (!X || !T) return mfail(m, HCU_INVALID_ARG, "null argument");
  if (!(lr > 0)) return mfail(m, HCU_INVALID_ARG, "learning rate must be positive");
  s = loss_and_grad(*m, X, T, idx, batch, loss);
  if (s != HCU_OK) return s;
  ++m->step;
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = (float)(1.0 - std::pow(0.9, m->step)), bc2 = (float)(1.0 - std::pow(0.999, m->step));
  k_adam<<<(unsigned)((m->np + 255) / 256), 256, 0, m->stream>>>(m->P, m->G, m->Mm, m->Vv, m->np, lr, b1, b2, 1e-8f,
                                                                 bc1, bc2);
  MLP_HIP(m, hipGetLastError());
  m->bf16_dirty = true;
  if (!loss) MLP_HIP(m, hipStreamSynchronize(m->stream));
  return HCU_OK;
}

hcu_status hcu_descriptor(hcu_ctx* ctx, float* desc, int* frame) {
  if (!ctx || !desc || !frame) return HCU_INVALID_ARG;
  Ctx& c = *ctx;
  if (!c.bound) return HCU_NOT_BOUND;
  if (c.hub_atoms.empty()) return HCU_OK;
  if (descriptor_scratch_bytes(c) > sizeof(double) * 16384 &&
      descriptor_scratch_bytes(c) > sizeof(double) * 8 * (size_t)c.p.natom) {
    c.err = "too many atoms for the descriptor scratch";
    return HCU_INVALID_ARG;
  }
  return run_descriptor(c, desc, frame);
}

hcu_status hcu_shell_density(hcu_ctx* ctx, double* out) {
  if (!ctx || !out) return HCU_INVALID_ARG;
  Ctx& c = *ctx;
  if (!c.bound) return HCU_NOT_BOUND;
  if (!c.have_results) {
    c.err = "no density yet";
    return HCU_INVALID_ARG;
  }
  const int nh = (int)c.hub_atoms.size();
  if (nh == 0) return HCU_OK;
  hcu_status st = compute_density(c);
  if (st != HCU_OK) return st;
  int nchunks = std::max(1, std::min(64, 16000 / (2 * kNShell * nh + 1)));
  // scratch in d_red: site positions then partials
  double* d_sites = c.d_red;
  double* d_part = c.d_red + 3 * nh + 1;
  if ((size_t)(3 * nh + 1 + (size_t)nh * nchunks * 2 * kNShell) > 16384) {
    c.err = "too many Hubbard sites for the shell scratch";
    return HCU_INVALID_ARG;
  }
  std::vector<double> sp(3 * nh);
  for (int h = 0; h < nh; ++h)
    for (int a = 0; a < 3; ++a) sp[3 * h + a] = c.pos[3 * c.hub_atoms[h] + a];
  HCU_HIP(hipMemcpyAsync(d_sites, sp.data(), sizeof(double) * 3 * nh, hipMemcpyHostToDevice, c.stream));
  int ni[3];
  image_counts(c, kShellHi + 8 * kGw, ni);
  dim3 grid(nchunks, nh);
  k_shells<<<grid, 256, 0, c.stream>>>(c.d_rho, c.p.nspin, c.nd, c.p.n[0], c.p.n[1], c.h[0], c.h[1], c.h[2],
                                       c.p.L[0], c.p.L[1], c.p.L[2], ni[0], ni[1], ni[2], d_sites, nchunks, d_part);
  HCU_HIP(hipGetLastError());
  std::vector<double> part((size_t)nh * nchunks * 2 * kNShell);
  HCU_HIP(hipMemcpyAsync(part.data(), d_part, sizeof(double) * part.size(), hipMemcpyDeviceToHost, c.stream));
  HCU_HIP(hipStreamSynchronize(c.stream));
  for (int h = 0; h < nh; ++h)
    for (int k = 0; k < kNShell; ++k) {
      double num = 0, den = 0;
      for (int ch = 0; ch < nchunks; ++ch) {
        num += part[((size_t)h * nchunks + ch) * 2 * kNShell + k];
        den += part[((size_t)h * nchunks + ch) * 2 * kNShell + kNShell + k];
      }
      out[h * kNShell + k] = den > 0 ? num / den : 0.0;
    }
  return HCU_OK;
}

hcu_status hcu_site_targets(hcu_ctx* ctx, float* out) {
  if (!ctx || !out) return HCU_INVALID_ARG;
  Ctx& c = *ctx;
  if (!c.bound) return HCU_NOT_BOUND;
  if (!c.have_results) {
    c.err = "no converged occupations yet";
    return HCU_INVALID_ARG;
  }
  const int nh = (int)c.hub_atoms.size();
  if (nh == 0) return HCU_OK;
  for (int h = 0; h < nh; ++h)
    if (c.hub_l[h] != 2) {
      c.err = "site targets cover d (l = 2) manifolds only";
      return HCU_INVALID_ARG;
    }
  std::vector<int> flags(nh);
  hcu_status s = run_descriptor(c, reinterpret_cast<float*>(c.d_vec), flags.data());
  if (s != HCU_OK) return s;
  std::vector<double> shells((size_t)nh * kNShell);
  s = hcu_shell_density(ctx, shells.data());
  if (s != HCU_OK) return s;
  for (int h = 0; h < nh; ++h) {
    double D[5][5];
    for (int i = 0; i < 5; ++i)
      for (int j = 0; j < 5; ++j) {
        double v = 0;
        for (int sp = 0; sp < c.p.nspin; ++sp) v += c.D_out[((size_t)sp * nh + h) * 25 + i * 5 + j];
        D[i][j] = v / c.p.nspin;
      }
    double Dl[5][5];
    if (flags[h]) {   // D_loc = M D M^T
      double T1[5][5];
      for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) {
          double acc = 0;
          for (int k = 0; k < 5; ++k) acc += D[i][k] * kFrame[j][k];
          T1[i][j] = acc;
        }
      for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) {
          double acc = 0;
          for (int k = 0; k < 5; ++k) acc += kFrame[i][k] * T1[k][j];
          Dl[i][j] = acc;
        }
    } else {
      std::memcpy(Dl, D, sizeof(Dl));
    }
    float* o = out + (size_t)h * 2 * kNShell;
    int t = 0;
    for (int i = 0; i < 5; ++i)
      for (int j = i; j < 5; ++j) o[t++] = (float)(0.5 * (Dl[i][j] + Dl[j][i]));
    for (int k = 0; k < kNShell; ++k) o[kNShell + k] = (float)shells[(size_t)h * kNShell + k];
  }
  return HCU_OK;
}

hcu_status hcu_mlp_guess(hcu_ctx* ctx, hcu_mlp* m, int bf16, float* outputs) {
  if (!ctx || !m) return HCU_INVALID_ARG;
  Ctx& c = *ctx;
  if (!c.bound) return HCU_NOT_BOUND;
  const int nh = (int)c.hub_atoms.size();
  if (nh == 0) return HCU_OK;
  hcu_status s = mlp_check(m, nh);
  if (s != HCU_OK) return s;
  if (m->dims[0] != kNG * c.p.nspecies) return mfail(m, HCU_INVALID_ARG, "MLP input width != 32 x species");
  if (m->dims[m->nl] < 15) return mfail(m, HCU_INVALID_ARG, "MLP needs at least 15 outputs");
  if (c.hub_l.size() != (size_t)nh) return mfail(m, HCU_INVALID_ARG, "internal: Hubbard table");
  for (int h = 0; h < nh; ++h)
    if (c.hub_l[h] != 2) return mfail(m, HCU_INVALID_ARG, "the learned guess covers d (l = 2) manifolds only");
  std::vector<int> flags(nh);
  s = hcu_descriptor(ctx, m->Xin, flags.data());
  if (s != HCU_OK) return s;
  const int no = m->dims[m->nl];
  float* Y = m->gB;   // device staging
  s = forward_out(*m, m->Xin, nh, Y, bf16);
  if (s != HCU_OK) return s;
  std::vector<float> y((size_t)nh * no);
  MLP_HIP(m, hipMemcpyAsync(y.data(), Y, sizeof(float) * y.size(), hipMemcpyDeviceToHost, m->stream));
  MLP_HIP(m, hipStreamSynchronize(m->stream));
  std::vector<double> D((size_t)c.p.nspin * nh * 25);
  for (int h = 0; h < nh; ++h) {
    double Dh[5][5];
    occupation_from_output(y.data() + (size_t)h * no, flags[h], Dh);
    for (int sp = 0; sp < c.p.nspin; ++sp)
      for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) D[((size_t)sp * nh + h) * 25 + i * 5 + j] = Dh[i][j];
  }
  if (outputs) std::memcpy(outputs, y.data(), sizeof(float) * y.size());
  return hcu_set_hubbard_occupation(ctx, D.data());
}

}  // extern "C"
