// Density-dependent part of the Hamiltonian and the mixing of the density
// (Sec. II.B: the ground state is found by Chebyshev-filtered subspace
// iteration with real-space preconditioned Pulay mixing; the coefficients
// found for the density also mix the occupation matrices).
//
//   V = V_loc + V_H[rho_in] + V_x[rho_in]
//   -Delta_h V_H = 4 pi (rho - <rho>)   (the kinetic term's order-2 n0
//       finite-difference Laplacian on the periodic grid; diagonal in plane
//       waves, so solved exactly in Fourier space with the stencil's symbol
//       lambda(G) = sum_a 2 (k_a0 + 2 sum_p k_ap cos(2 pi p m_a / n_a)),
//       k_ap the kinetic weights; lambda(0) = 0 is the neutralising background)
//   V_x = -(3 rho / pi)^(1/3), e_x = -(3/4)(3/pi)^(1/3) rho^(4/3)  (LDA exchange)
//   E_H = 1/2 int rho V_H = dV / (2 nd) sum_G 4 pi |rho^(G)|^2 / lambda(G)
//   F  += -int rho_out (V_H + V_x)[rho_in] + E_H[rho_out] + E_x[rho_out]
//
// Mixing (one Pulay step on rho): window of the last h+1 input densities x_i
// and residuals f_i = rho_out,i - x_i; gamma minimises |f - dF gamma| with
// dF_j = f_{j+1} - f_j; rho_bar = x - dX gamma, f_bar = f - dF gamma;
//   rho_in <- rho_bar + beta P f_bar,   P = (-Delta_h)(-Delta_h + k0^2)^-1
// (Kerker), the G = 0 coefficient set so that the cell holds N_e electrons.
// The m x m normal equations of gamma are formed on the device and solved on
// the host (m <= 8).
#include "common.h"

#include <hipfft/hipfft.h>

#include <cmath>

namespace hcu {
namespace {

constexpr int kHxThreads = 256;
constexpr int kHxBlocks = 512;            // reduction partials per quantity
constexpr int kHxMaxQ = 48;               // quantities of one reduction (Gram of 8 + rhs)

struct HxPtrs { const double* p[kHxcWindow]; };
struct HxGam { double g[kHxcWindow]; };

__device__ inline double hx_block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  return r;
}

// lambda(G) of the half spectrum entry q = kx + (n1/2+1) (ky + n2 kz), its
// Hermitian weight (2 for the entries standing for a conjugate pair too)
__device__ inline double hx_symbol(const double* sym, int n1, int n2, int64_t q, double* wgt) {
  const int nh = n1 / 2 + 1;
  const int kx = (int)(q % nh);
  const int ky = (int)((q / nh) % n2);
  const int kz = (int)(q / ((int64_t)nh * n2));
  if (wgt) *wgt = (kx == 0 || (2 * kx == n1)) ? 1.0 : 2.0;
  if (q == 0) return 0.0;
  return sym[kx] + sym[nh + ky] + sym[nh + n2 + kz];
}

__device__ inline double hx_vx(double r) { return r > 0 ? -cbrt(0.954929658551372014613 * r) : 0.0; }   // 3/pi

// partial sums: [0] rho_out (V - V_loc), [1] rho_out^(4/3), [2] (rho_out - rho_in)^2
__global__ void k_hx_grid_sums(const double* __restrict__ ro, const double* __restrict__ ri,
                               const double* __restrict__ V, const double* __restrict__ Vl, int64_t nd,
                               double* part) {
  __shared__ double sh[kHxThreads / 64];
  double s0 = 0, s1 = 0, s2 = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += (int64_t)gridDim.x * blockDim.x) {
    const double r = ro[i];
    s0 += r * (V[i] - Vl[i]);
    const double rp = r > 0 ? r : 0.0;
    s1 += rp * cbrt(rp);
    const double d = r - ri[i];
    s2 += d * d;
  }
  s0 = hx_block_sum(s0, sh);
  s1 = hx_block_sum(s1, sh);
  s2 = hx_block_sum(s2, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s0;
    part[gridDim.x + blockIdx.x] = s1;
    part[2 * gridDim.x + blockIdx.x] = s2;
  }
}

// partial sums of w |S(G)|^2 / lambda(G) over G != 0
__global__ void k_hx_spec_energy(const double2* __restrict__ S, const double* __restrict__ sym, int n1, int n2,
                                 int64_t nc, double* part) {
  __shared__ double sh[kHxThreads / 64];
  double s = 0;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nc; q += (int64_t)gridDim.x * blockDim.x) {
    double w;
    const double lam = hx_symbol(sym, n1, n2, q, &w);
    if (lam > 0) {
      const double2 v = S[q];
      s += w * (v.x * v.x + v.y * v.y) / lam;
    }
  }
  s = hx_block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out[q] = sum of the kHxBlocks partials of quantity q (one workgroup each)
__global__ void k_hx_final(const double* __restrict__ part, int np, double* out) {
  __shared__ double sh[kHxThreads / 64];
  double s = 0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[(int64_t)blockIdx.x * np + i];
  s = hx_block_sum(s, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// the newest window entry: x = rho_in, f = rho_out - rho_in
__global__ void k_hx_push(const double* __restrict__ ro, const double* __restrict__ ri, double* x, double* f,
                          int64_t nd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nd) return;
  const double r = ri[i];
  x[i] = r;
  f[i] = ro[i] - r;
}

// Normal equations of the Pulay least squares: G_jk = dF_j . dF_k (j <= k,
// row-major upper triangle), then b_j = dF_j . f_m; dF_j = f_{j+1} - f_j.
template <int M>
__global__ void k_hx_gram(HxPtrs f, int64_t nd, double* part) {
  __shared__ double sh[kHxThreads / 64];
  constexpr int NQ = M * (M + 1) / 2 + M;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += (int64_t)gridDim.x * blockDim.x) {
    double v[M + 1];
#pragma unroll
    for (int j = 0; j <= M; ++j) v[j] = f.p[j][i];
    double d[M];
#pragma unroll
    for (int j = 0; j < M; ++j) d[j] = v[j + 1] - v[j];
    int q = 0;
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
      for (int k = j; k < M; ++k) acc[q++] += d[j] * d[k];
#pragma unroll
    for (int j = 0; j < M; ++j) acc[q++] += d[j] * v[M];
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double s = hx_block_sum(acc[q], sh);
    if (threadIdx.x == 0) part[(int64_t)q * gridDim.x + blockIdx.x] = s;
  }
}

// rho_bar = x_m - sum_j g_j (x_{j+1} - x_j), f_bar likewise
__global__ void k_hx_combine(HxPtrs x, HxPtrs f, HxGam g, int m, int64_t nd, double* rb, double* fb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nd) return;
  double sx = 0, sf = 0;
  for (int j = 0; j < m; ++j) {
    sx += g.g[j] * (x.p[j + 1][i] - x.p[j][i]);
    sf += g.g[j] * (f.p[j + 1][i] - f.p[j][i]);
  }
  rb[i] = x.p[m][i] - sx;
  fb[i] = f.p[m][i] - sf;
}

// Fourier side of the mixing step and of the Hartree solve, in place:
// A <- rho_in^ = A + beta P(G) B (G = 0: g0), B <- V_H^ = 4 pi rho_in^ / lambda.
// With B == nullptr only the Hartree part: A <- 4 pi A / lambda.
__global__ void k_hx_spectrum(double2* A, double2* B, const double* __restrict__ sym, int n1, int n2, int64_t nc,
                              double beta, double k0sq, double g0) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc) return;
  const double lam = hx_symbol(sym, n1, n2, q, nullptr);
  const double2 a = A[q];
  double2 r = a;
  if (B) {
    const double2 b = B[q];
    const double p = lam > 0 ? lam / (lam + k0sq) : 0.0;
    r.x = a.x + beta * p * b.x;
    r.y = a.y + beta * p * b.y;
    if (q == 0) { r.x = g0; r.y = 0.0; }
  }
  const double s = lam > 0 ? 4.0 * M_PI / lam : 0.0;
  const double2 vh = make_double2(s * r.x, s * r.y);
  if (B) { A[q] = r; B[q] = vh; }
  else A[q] = vh;
}

// rho_in = rin_raw / nd (when given); V = V_loc + vh_raw / nd + V_x(rho_in)
__global__ void k_hx_assemble(const double* __restrict__ rin_raw, const double* __restrict__ vh_raw, double inv_nd,
                              const double* __restrict__ Vl, double* rho_in, double* V, float* Vf, int64_t nd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nd) return;
  double r;
  if (rin_raw) { r = rin_raw[i] * inv_nd; rho_in[i] = r; }
  else r = rho_in[i];
  const double v = Vl[i] + vh_raw[i] * inv_nd + hx_vx(r);
  V[i] = v;
  if (Vf) Vf[i] = (float)v;
}

__global__ void k_hx_fill(double* x, double v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

hcu_status fail(Ctx& c, hcu_status s, const std::string& msg) {
  c.err = msg;
  return s;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kHxThreads - 1) / kHxThreads); }

#define HCU_FFT(call)                                                              \
  do {                                                                             \
    hipfftResult r_ = (call);                                                      \
    if (r_ != HIPFFT_SUCCESS) return fail(c, HCU_DEVICE, "hipFFT error " + std::to_string((int)r_) + \
                                          " at " + __FILE__ + ":" + std::to_string(__LINE__));      \
  } while (0)

hipfftHandle plan(const Ctx& c, int i) { return reinterpret_cast<hipfftHandle>(c.hxc_plan[i]); }

hcu_status fft_r2c(Ctx& c, double* in, double* out) {
  HCU_FFT(hipfftSetStream(plan(c, 0), c.stream));
  HCU_FFT(hipfftExecD2Z(plan(c, 0), in, reinterpret_cast<hipfftDoubleComplex*>(out)));
  return HCU_OK;
}
// (the complex input is overwritten)
hcu_status fft_c2r(Ctx& c, double* in, double* out) {
  HCU_FFT(hipfftSetStream(plan(c, 1), c.stream));
  HCU_FFT(hipfftExecZ2D(plan(c, 1), reinterpret_cast<hipfftDoubleComplex*>(in), out));
  return HCU_OK;
}

// gamma = argmin |f - dF gamma| from the normal equations G gamma = b
// (symmetric Jacobi eigensolve; directions with eigenvalues below 1e-12 of
// the largest are dropped: the minimum-norm solution on the rest)
std::vector<double> pulay_solve(const std::vector<double>& G, const std::vector<double>& b, int m) {
  std::vector<double> A = G, Vv(m * m, 0.0);
  for (int i = 0; i < m; ++i) Vv[i * m + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        tot += A[i * m + j] * A[i * m + j];
        if (i != j) off += A[i * m + j] * A[i * m + j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = A[p * m + q];
        if (apq == 0.0) continue;
        const double th = (A[q * m + q] - A[p * m + p]) / (2 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1));
        const double cs = 1 / std::sqrt(t * t + 1), sn = t * cs;
        for (int k = 0; k < m; ++k) {   // A <- J^T A J
          const double akp = A[k * m + p], akq = A[k * m + q];
          A[k * m + p] = cs * akp - sn * akq;
          A[k * m + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < m; ++k) {
          const double apk = A[p * m + k], aqk = A[q * m + k];
          A[p * m + k] = cs * apk - sn * aqk;
          A[q * m + k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < m; ++k) {
          const double vkp = Vv[k * m + p], vkq = Vv[k * m + q];
          Vv[k * m + p] = cs * vkp - sn * vkq;
          Vv[k * m + q] = sn * vkp + cs * vkq;
        }
      }
  }
  double lmax = 0;
  for (int i = 0; i < m; ++i) lmax = std::max(lmax, A[i * m + i]);
  std::vector<double> g(m, 0.0);
  for (int e = 0; e < m; ++e) {
    const double l = A[e * m + e];
    if (!(l > 1e-12 * lmax)) continue;
    double vb = 0;
    for (int i = 0; i < m; ++i) vb += Vv[i * m + e] * b[i];
    for (int i = 0; i < m; ++i) g[i] += Vv[i * m + e] * vb / l;
  }
  return g;
}

}  // namespace

size_t hxc_spectrum_elems(const Ctx& c) { return (size_t)(c.p.n[0] / 2 + 1) * c.p.n[1] * c.p.n[2]; }
size_t hxc_partial_elems() { return (size_t)kHxMaxQ * kHxBlocks + 64; }

// V from d_rho_in and d_Vloc (d_V, and d_Vf for FP32 blocks)
hcu_status hxc_refresh_potential(Ctx& c) {
  const int64_t nd = c.nd, nc = (int64_t)hxc_spectrum_elems(c);
  double* S = c.d_hspec;
  hcu_status s = fft_r2c(c, c.d_rho_in, S);
  if (s != HCU_OK) return s;
  k_hx_spectrum<<<blocks_for(nc), kHxThreads, 0, c.stream>>>((double2*)S, nullptr, c.d_hsym, c.p.n[0], c.p.n[1], nc,
                                                              0.0, 0.0, 0.0);
  HCU_HIP(hipGetLastError());
  s = fft_c2r(c, S, c.d_hbar);
  if (s != HCU_OK) return s;
  k_hx_assemble<<<blocks_for(nd), kHxThreads, 0, c.stream>>>(nullptr, c.d_hbar, 1.0 / (double)nd, c.d_Vloc,
                                                              c.d_rho_in, c.d_V, c.mixed ? c.d_Vf : nullptr, nd);
  HCU_HIP(hipGetLastError());
  return HCU_OK;
}

// Uniform input density N_e / Omega and its potential; the mixing window is emptied.
hcu_status hxc_reset_density(Ctx& c) {
  const double omega = c.p.L[0] * c.p.L[1] * c.p.L[2];
  k_hx_fill<<<blocks_for(c.nd), kHxThreads, 0, c.stream>>>(c.d_rho_in, c.p.nelec / omega, c.nd);
  HCU_HIP(hipGetLastError());
  c.hxc_slots.clear();
  c.hxc_have_rho = true;
  return hxc_refresh_potential(c);
}

// After the structure tables are (re)built: symbol tables and FFT plans on
// the first call, the uniform density if there is none yet, the potential.
hcu_status hxc_after_structure(Ctx& c) {
  if (!c.hxc) return HCU_OK;
  const int n1 = c.p.n[0], n2 = c.p.n[1], n3 = c.p.n[2], nh = n1 / 2 + 1;
  StencilCoef sc;
  fill_stencil_coef(c, 0, sc);
  std::vector<double> sym(nh + n2 + n3);
  const int nn[3] = {n1, n2, n3}, off[3] = {0, nh, nh + n2}, cnt[3] = {nh, n2, n3};
  for (int a = 0; a < 3; ++a)
    for (int m = 0; m < cnt[a]; ++m) {
      double v = sc.kin[a][0];
      for (int p = 1; p <= c.p.n0; ++p) v += 2.0 * sc.kin[a][p] * std::cos(2.0 * M_PI * p * m / nn[a]);
      sym[off[a] + m] = m == 0 ? 0.0 : 2.0 * v;   // the weights sum to zero at m = 0
    }
  HCU_HIP(hipMemcpyAsync(c.d_hsym, sym.data(), sizeof(double) * sym.size(), hipMemcpyHostToDevice, c.stream));
  if (!c.hxc_plan[0]) {
    hipfftHandle p0 = nullptr, p1 = nullptr;
    HCU_FFT(hipfftPlan3d(&p0, n3, n2, n1, HIPFFT_D2Z));
    c.hxc_plan[0] = p0;
    HCU_FFT(hipfftPlan3d(&p1, n3, n2, n1, HIPFFT_Z2D));
    c.hxc_plan[1] = p1;
  }
  HCU_HIP(hipStreamSynchronize(c.stream));   // sym is released on return
  if (!c.hxc_have_rho) return hxc_reset_density(c);
  return hxc_refresh_potential(c);
}

void hxc_destroy(Ctx& c) {
  for (int i = 0; i < 2; ++i)
    if (c.hxc_plan[i]) { hipfftDestroy(reinterpret_cast<hipfftHandle>(c.hxc_plan[i])); c.hxc_plan[i] = nullptr; }
}

// Energies of the output density in d_rho (after the density kernel):
// E_H[rho_out], E_x[rho_out], -int rho_out (V_H + V_x)[rho_in], and the
// density residual sqrt(dV sum (rho_out - rho_in)^2) / N_e.
hcu_status hxc_energies(Ctx& c) {
  const int64_t nd = c.nd, nc = (int64_t)hxc_spectrum_elems(c);
  double* part = c.d_hpart;
  double* out = c.d_hpart + (size_t)kHxMaxQ * kHxBlocks;
  k_hx_grid_sums<<<kHxBlocks, kHxThreads, 0, c.stream>>>(c.d_rho, c.d_rho_in, c.d_V, c.d_Vloc, nd, part);
  HCU_HIP(hipGetLastError());
  HCU_HIP(hipMemcpyAsync(c.d_hbar, c.d_rho, sizeof(double) * nd, hipMemcpyDeviceToDevice, c.stream));
  hcu_status s = fft_r2c(c, c.d_hbar, c.d_hspec);
  if (s != HCU_OK) return s;
  k_hx_spec_energy<<<kHxBlocks, kHxThreads, 0, c.stream>>>((const double2*)c.d_hspec, c.d_hsym, c.p.n[0], c.p.n[1],
                                                            nc, part + 3 * kHxBlocks);
  HCU_HIP(hipGetLastError());
  k_hx_final<<<4, kHxThreads, 0, c.stream>>>(part, kHxBlocks, out);
  HCU_HIP(hipGetLastError());
  double h[4];
  HCU_HIP(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, c.stream));
  HCU_HIP(hipStreamSynchronize(c.stream));
  const double dv = c.dv;
  c.en.E_H = dv / (2.0 * (double)nd) * 4.0 * M_PI * h[3];
  c.en.E_x = -0.75 * std::cbrt(3.0 / M_PI) * dv * h[1];
  c.en.e_hxc = -dv * h[0] + c.en.E_H + c.en.E_x;
  c.hxc_res = std::sqrt(dv * h[2]) / c.p.nelec;
  return HCU_OK;
}

// One Pulay step on the density (window of at most hist + 1 entries) with the
// Kerker-preconditioned residual step; installs the new rho_in and V and
// returns the coefficients gamma (oldest difference first).
hcu_status hxc_mix(Ctx& c, int hist, double beta, double k0, std::vector<double>& gamma) {
  const int64_t nd = c.nd, nc = (int64_t)hxc_spectrum_elems(c);
  if (hist + 1 > kHxcWindow) return fail(c, HCU_INVALID_ARG, "density mixing history too long");
  // newest entry: reuse the oldest slot once the window is full
  int slot;
  if ((int)c.hxc_slots.size() >= hist + 1) {
    slot = c.hxc_slots.front();
    c.hxc_slots.erase(c.hxc_slots.begin());
  } else {
    std::vector<int> used(kHxcWindow, 0);
    for (int u : c.hxc_slots) used[u] = 1;
    slot = 0;
    while (used[slot]) ++slot;
  }
  c.hxc_slots.push_back(slot);
  k_hx_push<<<blocks_for(nd), kHxThreads, 0, c.stream>>>(c.d_rho, c.d_rho_in, c.d_hx + (size_t)slot * nd,
                                                          c.d_hf + (size_t)slot * nd, nd);
  HCU_HIP(hipGetLastError());
  const int m = (int)c.hxc_slots.size() - 1;
  HxPtrs X{}, F{};
  for (int i = 0; i <= m; ++i) {
    X.p[i] = c.d_hx + (size_t)c.hxc_slots[i] * nd;
    F.p[i] = c.d_hf + (size_t)c.hxc_slots[i] * nd;
  }
  gamma.assign(m, 0.0);
  if (m > 0) {
    double* part = c.d_hpart;
    double* out = c.d_hpart + (size_t)kHxMaxQ * kHxBlocks;
    const int nq = m * (m + 1) / 2 + m;
    switch (m) {
      case 1: k_hx_gram<1><<<kHxBlocks, kHxThreads, 0, c.stream>>>(F, nd, part); break;
      case 2: k_hx_gram<2><<<kHxBlocks, kHxThreads, 0, c.stream>>>(F, nd, part); break;
      case 3: k_hx_gram<3><<<kHxBlocks, kHxThreads, 0, c.stream>>>(F, nd, part); break;
      case 4: k_hx_gram<4><<<kHxBlocks, kHxThreads, 0, c.stream>>>(F, nd, part); break;
      case 5: k_hx_gram<5><<<kHxBlocks, kHxThreads, 0, c.stream>>>(F, nd, part); break;
      case 6: k_hx_gram<6><<<kHxBlocks, kHxThreads, 0, c.stream>>>(F, nd, part); break;
      case 7: k_hx_gram<7><<<kHxBlocks, kHxThreads, 0, c.stream>>>(F, nd, part); break;
      default: k_hx_gram<8><<<kHxBlocks, kHxThreads, 0, c.stream>>>(F, nd, part); break;
    }
    HCU_HIP(hipGetLastError());
    k_hx_final<<<nq, kHxThreads, 0, c.stream>>>(part, kHxBlocks, out);
    HCU_HIP(hipGetLastError());
    std::vector<double> h(nq);
    HCU_HIP(hipMemcpyAsync(h.data(), out, sizeof(double) * nq, hipMemcpyDeviceToHost, c.stream));
    HCU_HIP(hipStreamSynchronize(c.stream));
    std::vector<double> G(m * m), b(m);
    int q = 0;
    for (int j = 0; j < m; ++j)
      for (int k = j; k < m; ++k) { G[j * m + k] = G[k * m + j] = h[q]; ++q; }
    for (int j = 0; j < m; ++j) b[j] = h[q++];
    for (double v : h)
      if (!std::isfinite(v)) return fail(c, HCU_NAN, "non-finite density residual");
    gamma = pulay_solve(G, b, m);
  }
  HxGam g{};
  for (int j = 0; j < m; ++j) g.g[j] = gamma[j];
  double* rb = c.d_hbar;
  double* fb = c.d_hbar + nd;
  k_hx_combine<<<blocks_for(nd), kHxThreads, 0, c.stream>>>(X, F, g, m, nd, rb, fb);
  HCU_HIP(hipGetLastError());
  double* SA = c.d_hspec;
  double* SB = c.d_hspec + 2 * nc;
  hcu_status s = fft_r2c(c, rb, SA);
  if (s != HCU_OK) return s;
  s = fft_r2c(c, fb, SB);
  if (s != HCU_OK) return s;
  const double omega = c.p.L[0] * c.p.L[1] * c.p.L[2];
  k_hx_spectrum<<<blocks_for(nc), kHxThreads, 0, c.stream>>>((double2*)SA, (double2*)SB, c.d_hsym, c.p.n[0], c.p.n[1],
                                                              nc, beta, k0 * k0, c.p.nelec / omega * (double)nd);
  HCU_HIP(hipGetLastError());
  s = fft_c2r(c, SA, rb);
  if (s != HCU_OK) return s;
  s = fft_c2r(c, SB, fb);
  if (s != HCU_OK) return s;
  k_hx_assemble<<<blocks_for(nd), kHxThreads, 0, c.stream>>>(rb, fb, 1.0 / (double)nd, c.d_Vloc, c.d_rho_in, c.d_V,
                                                              c.mixed ? c.d_Vf : nullptr, nd);
  HCU_HIP(hipGetLastError());
  return HCU_OK;
}

}  // namespace hcu
