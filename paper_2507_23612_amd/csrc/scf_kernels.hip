// Small FP64 kernels of the SCF step: Fermi level and occupations, Hubbard
// occupation matrices, Hubbard energy and free energy, density, and the
// vector helpers of the Lanczos bound.
//
// Occupations are Fermi-Dirac with one Fermi level for every spin and
// k-point (Eq. orbital_occup_ext uses occupations f_j(k) and a Brillouin-zone
// average).  D_I = sum_k w_k P F P^H (Eq. orbital_occup_ext),
// E_U = sum_sigma sum_I U/2 Tr(D - D^2) (Eq. E_U).
#include "common.h"

namespace hcu {

__device__ inline double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// ------------------------------------------------------------------ dot
// out2[0] = Re sum conj(x) y, out2[1] = Im; two deterministic stages.
template <typename T>
__global__ void k_dot_part(const T* __restrict__ x, const T* __restrict__ y, int64_t n, double* part) {
  __shared__ double sh[256];
  double re = 0, im = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    T p = mul_conj(y[i], x[i]);
    if constexpr (sizeof(T) == sizeof(typename real_of<T>::type)) re += (double)p;
    else { re += (double)p.re; im += (double)p.im; }
  }
  re = block_sum(re, sh);
  im = block_sum(im, sh);
  if (threadIdx.x == 0) { part[2 * blockIdx.x] = re; part[2 * blockIdx.x + 1] = im; }
}
__global__ void k_dot_final(const double* part, int np, double* out2) {
  __shared__ double sh[256];
  double re = 0, im = 0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) { re += part[2 * i]; im += part[2 * i + 1]; }
  re = block_sum(re, sh);
  im = block_sum(im, sh);
  if (threadIdx.x == 0) { out2[0] = re; out2[1] = im; }
}

template <typename T>
void launch_dot(const Ctx& c, const T* x, const T* y, int64_t n, double* out2, hipStream_t st) {
  const int np = 256;
  k_dot_part<T><<<np, 256, 0, st>>>(x, y, n, c.d_red);
  k_dot_final<<<1, 256, 0, st>>>(c.d_red, np, out2);
}

// y = a x + b y (a complex, b real)
template <typename T>
__global__ void k_axpby(T* y, const T* x, double are, double aim, double b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  using R = typename real_of<T>::type;
  T a = make_scalar<T>(are, aim);
  T v = (R)b * y[i];
  if (x) v += a * x[i];
  y[i] = v;
}
template <typename T>
void launch_axpby(const Ctx& c, T* y, const T* x, double a_re, double a_im, double b, int64_t n, hipStream_t st) {
  (void)c;
  k_axpby<T><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(y, x, a_re, a_im, b, n);
}

template <typename T>
__global__ void k_scale_copy(T* dst, const T* src, double s, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (typename real_of<T>::type)s * src[i];
}
template <typename T>
void launch_scale_copy(T* dst, const T* src, double s, int64_t n, hipStream_t st) {
  k_scale_copy<T><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(dst, src, s, n);
}

// eigenvectors (double, or interleaved double complex) -> block precision
template <typename T>
__global__ void k_convert_c(const double* C, T* Cb, int64_t nn, int cp) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  Cb[i] = cp ? make_scalar<T>(C[2 * i], C[2 * i + 1]) : make_scalar<T>(C[i], 0.0);
}
template <typename T>
void launch_convert_c(const double* C, T* Cb, int n, int cplx_, hipStream_t st) {
  int64_t nn = (int64_t)n * n;
  k_convert_c<T><<<(unsigned)((nn + 255) / 256), 256, 0, st>>>(C, Cb, nn, cplx_);
}

// ------------------------------------------------------------------ Fermi level
// lam, occ: [nsk][ns]; kw per sk (k weight).  Bisection on the electron count
// with bracket [min - 1, max + 1] until the bracket stops shrinking.
// scal[0] = mu, scal[1] = e_band, scal[4] = kT * S.
__global__ void k_fermi(const double* __restrict__ lam, double* __restrict__ occ, const double* __restrict__ kw_sk,
                        int nsk, int ns, double nelec, double kT, double gs, double* scal) {
  __shared__ double sh[256];
  const int tot = nsk * ns;
  double lo, hi;
  {
    double mn = 1e300, mx = -1e300;
    for (int i = threadIdx.x; i < tot; i += blockDim.x) { mn = fmin(mn, lam[i]); mx = fmax(mx, lam[i]); }
    sh[threadIdx.x] = mn;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) { if (threadIdx.x < s) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + s]); __syncthreads(); }
    mn = sh[0];
    __syncthreads();
    sh[threadIdx.x] = mx;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) { if (threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]); __syncthreads(); }
    mx = sh[0];
    __syncthreads();
    lo = mn - 1.0;
    hi = mx + 1.0;
  }
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    double cnt = 0;
    for (int i = threadIdx.x; i < tot; i += blockDim.x) cnt += kw_sk[i / ns] / (1.0 + exp((lam[i] - mid) / kT));
    cnt = gs * block_sum(cnt, sh);
    if (cnt < nelec) lo = mid; else hi = mid;
  }
  const double mu = 0.5 * (lo + hi);
  double eb = 0, ent = 0;
  for (int i = threadIdx.x; i < tot; i += blockDim.x) {
    const double f = 1.0 / (1.0 + exp((lam[i] - mu) / kT));
    occ[i] = f;
    const double w = kw_sk[i / ns];
    eb += w * f * lam[i];
    if (f > 0.0 && f < 1.0) ent += w * (f * log(f) + (1.0 - f) * log(1.0 - f));
  }
  eb = gs * block_sum(eb, sh);
  ent = -gs * block_sum(ent, sh);
  if (threadIdx.x == 0) { scal[0] = mu; scal[1] = eb; scal[4] = kT * ent; }
}

void launch_fermi(const Ctx& c, hipStream_t st) {
  const int nsk = c.p.nspin * c.p.nk;
  double* kw_sk = c.d_scal + 64;     // filled by the driver
  const double gs = c.p.nspin == 1 ? 2.0 : 1.0;
  k_fermi<<<1, 256, 0, st>>>(c.d_lam, c.d_occ, kw_sk, nsk, c.p.ns, c.p.nelec, c.p.kT, gs, c.d_scal);
}

// ------------------------------------------------------------------ D
// D[spin][h] (+)= w_k sum_s f_s P[s][j0+m] conj(P[s][j0+m']) (real part kept).
template <typename T>
__global__ void k_occmat(const T* __restrict__ PX, const double* __restrict__ occ, const BlockDesc* __restrict__ blocks,
                         const int* __restrict__ hub_blocks, int ns, int nproj, double w, int accumulate,
                         double* __restrict__ D) {
  __shared__ double sh[256];
  const BlockDesc b = blocks[hub_blocks[blockIdx.x]];
  const int nm = b.nm;
  double* Dh = D + (int64_t)blockIdx.x * 25;
  for (int e = 0; e < nm * nm; ++e) {
    const int m = e / nm, mp = e % nm;
    double acc = 0;
    for (int s = threadIdx.x; s < ns; s += blockDim.x) {
      T pm = PX[(int64_t)s * nproj + b.j0 + m], pmp = PX[(int64_t)s * nproj + b.j0 + mp];
      T pr = mul_conj(pm, pmp);
      double re;
      if constexpr (sizeof(T) == sizeof(typename real_of<T>::type)) re = (double)pr;
      else re = (double)pr.re;
      acc += occ[s] * re;
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) Dh[m * 5 + mp] = (accumulate ? Dh[m * 5 + mp] : 0.0) + w * acc;
  }
}

template <typename T>
void launch_occupation_matrix(const Ctx& c, int spin, int ik, const T* PX, hipStream_t st) {
  const int nh = (int)c.hub_atoms.size();
  if (nh == 0) return;
  const int sk = sk_index(c, spin, ik);
  k_occmat<T><<<nh, 256, 0, st>>>(PX, c.d_occ + (int64_t)sk * c.p.ns, c.d_blocks, c.d_hub_blocks, c.p.ns, c.nproj,
                                  c.kw[ik], ik > 0 ? 1 : 0, c.d_D + (int64_t)spin * nh * 25);
}

// ------------------------------------------------------------------ energies
// Symmetrise D, then scal[2] = dc = sum Tr(M_in D_out), scal[3] = E_U, both
// counted twice for nspin = 1; scal[5] = F = e_band - dc + E_U - kT S.
__global__ void k_energies(double* D, const double* const* coup_by_spin, const BlockDesc* blocks,
                           const int* hub_blocks, const double* hubU, int nspin, int nh, double* scal) {
  if (threadIdx.x != 0) return;
  double dc = 0, eu = 0;
  for (int s = 0; s < nspin; ++s) {
    const double* coup = coup_by_spin[s];
    for (int h = 0; h < nh; ++h) {
      const BlockDesc b = blocks[hub_blocks[h]];
      const int nm = b.nm;
      double* d = D + ((int64_t)s * nh + h) * 25;
      for (int i = 0; i < nm; ++i)
        for (int j = i + 1; j < nm; ++j) {
          double v = 0.5 * (d[i * 5 + j] + d[j * 5 + i]);
          d[i * 5 + j] = v;
          d[j * 5 + i] = v;
        }
      const double* M = coup + b.coup_off;
      double tr = 0, tr2 = 0, trmd = 0;
      for (int i = 0; i < nm; ++i) {
        tr += d[i * 5 + i];
        for (int j = 0; j < nm; ++j) {
          tr2 += d[i * 5 + j] * d[j * 5 + i];
          trmd += M[i * nm + j] * d[j * 5 + i];
        }
      }
      eu += 0.5 * hubU[h] * (tr - tr2);
      dc += trmd;
    }
  }
  const double f = nspin == 1 ? 2.0 : 1.0;
  scal[2] = f * dc;
  scal[3] = f * eu;
  scal[5] = scal[1] - scal[2] + scal[3] - scal[4];
}

void launch_energies(const Ctx& c, const double* d_coup_ptrs, hipStream_t st) {
  const int nh = (int)c.hub_atoms.size();
  const int nsk = c.p.nspin * c.p.nk;
  const double* hubU = c.d_scal + 64 + nsk;   // filled by the driver
  const double* const* cps = reinterpret_cast<const double* const*>(c.d_scal + 64 + nsk + nh);
  (void)d_coup_ptrs;
  k_energies<<<1, 64, 0, st>>>(c.d_D, cps, c.d_blocks, c.d_hub_blocks, hubU, c.p.nspin, nh, c.d_scal);
}

// ------------------------------------------------------------------ density
template <typename T>
__global__ void k_density(const T* __restrict__ X, int64_t ld, int ns, const double* __restrict__ occ, double w,
                          int64_t nd, double* __restrict__ rho) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nd) return;
  double acc = 0;
  for (int s = 0; s < ns; ++s) acc += occ[s] * (double)abs2_(X[(int64_t)s * ld + p]);
  rho[p] += w * acc;
}

template <typename T>
void launch_density(const Ctx& c, const T* X, int64_t ld, const double* occ, double w, double* rho, hipStream_t st) {
  k_density<T><<<(unsigned)((c.nd + 255) / 256), 256, 0, st>>>(X, ld, c.p.ns, occ, w, c.nd, rho);
}

#define INST(T)                                                                                        \
  template void launch_dot<T>(const Ctx&, const T*, const T*, int64_t, double*, hipStream_t);         \
  template void launch_axpby<T>(const Ctx&, T*, const T*, double, double, double, int64_t, hipStream_t); \
  template void launch_scale_copy<T>(T*, const T*, double, int64_t, hipStream_t);                      \
  template void launch_convert_c<T>(const double*, T*, int, int, hipStream_t);                         \
  template void launch_occupation_matrix<T>(const Ctx&, int, int, const T*, hipStream_t);              \
  template void launch_density<T>(const Ctx&, const T*, int64_t, const double*, double, double*, hipStream_t);
INST(double)
INST(float)
INST(cplx<double>)
INST(cplx<float>)

}  // namespace hcu

namespace hcu {

// ---------------------------------------------------------------- Rayleigh-Ritz guards
// The projected problem Hs C = S C diag(lam) is handed to library routines
// (Cholesky, triangular solves, symmetric eigensolver) that must not see
// non-finite or half-factorised data.  Before the Cholesky factorisation:
// any non-finite entry of the upper triangles of S or Hs sets info[2] and
// replaces both matrices by the identity.  After it: a failed factorisation
// (info[0] != 0, S not positive definite) replaces the factor and Hs by the
// identity.  The library steps then run on harmless data and the host
// reports the recorded status.  One workgroup; n x n column-major, complex
// interleaved when cp = 2.
__device__ void set_identity(double* A, int n, int cp) {
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = threadIdx.x; e < nn; e += blockDim.x) {
    const int64_t i = e % n, j = e / n;
    A[cp * e] = i == j ? 1.0 : 0.0;
    if (cp == 2) A[cp * e + 1] = 0.0;
  }
}

__global__ __launch_bounds__(1024) void k_rr_guard_in(double* S, double* Hs, int n, int cp, int* info) {
  int bad = 0;
  const int64_t nn = (int64_t)n * n;
  for (int64_t e = threadIdx.x; e < nn; e += blockDim.x) {
    const int64_t i = e % n, j = e / n;
    if (i > j) continue;   // upper triangle only (what the factorisation reads)
    for (int h = 0; h < cp; ++h)
      if (!isfinite(S[cp * e + h]) || !isfinite(Hs[cp * e + h])) bad = 1;
  }
  bad = __syncthreads_or(bad);
  if (bad) {
    set_identity(S, n, cp);
    set_identity(Hs, n, cp);
  }
  if (threadIdx.x == 0) info[2] = bad;
}

__global__ __launch_bounds__(1024) void k_rr_guard_chol(double* U, double* Hs, int n, int cp, const int* info) {
  if (info[0] == 0) return;
  set_identity(U, n, cp);
  set_identity(Hs, n, cp);
}

void launch_rr_guard_in(double* S, double* Hs, int n, int cp, int* info, hipStream_t st) {
  launch_k(k_rr_guard_in, 1, 1024, 0, st, S, Hs, n, cp, info);
}
void launch_rr_guard_chol(double* U, double* Hs, int n, int cp, const int* info, hipStream_t st) {
  launch_k(k_rr_guard_chol, 1, 1024, 0, st, U, Hs, n, cp, info);
}

}  // namespace hcu
