// C ABI of the library: context, workspace, operator, Chebyshev filter,
// Rayleigh-Ritz pass, Lanczos bound and the SCF loop of real-space DFT+U
// (arXiv:2507.23612, Sec. II.B: ChFSI ground state, Pulay mixing of the
// occupation matrices, D updated every SCF iteration).
#include "common.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

using namespace hcu;


struct hcu_batch {
  std::vector<hcu_ctx*> m;
  std::string err;
};

namespace {

struct Bump {
  char* base;
  bool assign = true;   // false: only measure
  size_t off = 0;
  template <typename P>
  void take(P*& ptr, size_t bytes) {
    off = (off + 255) & ~size_t(255);
    if (assign) ptr = base ? reinterpret_cast<P*>(base + off) : nullptr;
    off += std::max<size_t>(bytes, 1);
  }
};

size_t esize(const Ctx& c) { return (c.mixed ? 4 : 8) * (c.any_complex ? 2 : 1); }

constexpr int kInfoPerBlock = 4;   // eigensolve status words per (spin, k): Cholesky, eigensolver, guard
constexpr size_t kBatchJobBytes = 1 << 20;   // stencil job records of one batched pass (~2900 jobs)
constexpr unsigned long long kPersistentMinItems = 4096;   // smaller batched launches use one workgroup per item

// Workspace layout.  Buffers whose size does not depend on the atom
// positions come first (orbitals, work blocks, small dense buffers), then the
// position-dependent tables (supports, bricks, function values), so that
// moving the atoms re-lays out only the tail and the orbitals stay in place.
// assign = false measures without touching the context's pointers.
size_t layout(Ctx& c, char* base, bool assign = true) {
  Bump b{base, assign};
  const size_t es = esize(c);
  const int nsk = c.p.nspin * c.p.nk;
  const int ns = c.p.ns;
  const int nh = (int)c.hub_atoms.size();
  const int cp = c.any_complex ? 2 : 1;
  // ---- position independent
  b.take(c.d_V, sizeof(double) * c.nd);
  if (c.mixed) b.take(c.d_Vf, sizeof(float) * c.nd);
  b.take(c.d_blocks, sizeof(BlockDesc) * c.blocks.size());
  b.take(c.d_nm_lists, sizeof(int) * c.blocks.size());
  b.take(c.d_hub_blocks, sizeof(int) * nh);
  std::vector<double*> coup(c.p.nspin, nullptr);
  for (int s = 0; s < c.p.nspin; ++s) b.take(coup[s], sizeof(double) * c.coup_size);
  std::vector<void*> X(nsk), v0(nsk), PX(nsk), W(3 * nsk), P(nsk), Q(nsk), PY(nsk);
  for (int i = 0; i < nsk; ++i) {
    b.take(X[i], es * (size_t)c.nd * ns);
    b.take(v0[i], es * (size_t)c.nd);
    b.take(PX[i], es * (size_t)ns * c.nproj);
  }
  for (int i = 0; i < nsk; ++i) {
    for (int w = 0; w < 3; ++w) b.take(W[3 * i + w], es * (size_t)c.nd * ns);
    b.take(P[i], es * (size_t)ns * c.nproj);
    b.take(Q[i], es * (size_t)ns * c.nproj);
    b.take(PY[i], es * (size_t)ns * c.nproj);
  }
  if (assign) {
    c.d_coup = coup;
    c.d_X = X; c.d_v0 = v0; c.d_PX = PX; c.d_W = W; c.d_P = P; c.d_Q = Q; c.d_PY = PY;
  }
  b.take(c.d_jobs, kBatchJobBytes);
  b.take(c.d_counters, sizeof(unsigned long long) * kNumXcd);
  const size_t part_elems = c.any_complex ? gram_partial_elems_c(ns, c.nd) : gram_partial_elems(ns, c.nd);
  if (assign) c.part_elems = part_elems;
  b.take(c.d_part, sizeof(double) * part_elems);
  b.take(c.d_tiles, sizeof(int2) * gram_tiles(ns, c.any_complex).size());
  b.take(c.d_S, sizeof(double) * (size_t)ns * ns * cp);
  b.take(c.d_Hs, sizeof(double) * (size_t)ns * ns * cp);
  b.take(c.d_C, sizeof(double) * (size_t)ns * ns * cp);
  b.take(c.d_Cb, es * (size_t)ns * ns);
  b.take(c.d_lam, sizeof(double) * (size_t)nsk * ns);
  b.take(c.d_occ, sizeof(double) * (size_t)nsk * ns);
  b.take(c.d_E, sizeof(double) * (size_t)ns * (c.any_complex ? 4 : 2));   // e, then tau (complex: 2 per entry)
  b.take(c.d_info, sizeof(int) * 4);
  std::vector<Ctx::RRSlot> slots((size_t)std::max(0, std::min(nsk, kRRLanes) - 1));
  for (size_t i = 0; i < slots.size(); ++i) {
    Ctx::RRSlot& r = slots[i];
    if (i < c.rr_slots.size()) r.blas = c.rr_slots[i].blas;
    b.take(r.part, sizeof(double) * part_elems);
    b.take(r.S, sizeof(double) * (size_t)ns * ns * cp);
    b.take(r.Hs, sizeof(double) * (size_t)ns * ns * cp);
    b.take(r.Cb, es * (size_t)ns * ns);
    b.take(r.E, sizeof(double) * (size_t)ns * (c.any_complex ? 4 : 2));
    b.take(r.info, sizeof(int) * 4);
  }
  if (assign) c.rr_slots = slots;
  b.take(c.d_D, sizeof(double) * (size_t)c.p.nspin * nh * 25);
  size_t red = std::max<size_t>(16384 * sizeof(double), sizeof(double) * 8 * (size_t)c.p.natom);
  red = std::max(red, sizeof(int) * c.blocks.size());
  b.take(c.d_red, red);
  b.take(c.d_scal, sizeof(double) * (64 + nsk + nh + c.p.nspin + 8));
  b.take(c.d_rho, sizeof(double) * (size_t)c.p.nspin * c.nd);
  b.take(c.d_vec, es * (size_t)c.nd * 4);
  b.take(c.d_lowC, sizeof(double) * 50 * (size_t)c.p.nk * nh);
  b.take(c.d_fproj, es * 13 * (size_t)ns * c.nproj);
  b.take(c.d_fsum, sizeof(double) * 650 * (size_t)nh);
  b.take(c.d_focc, sizeof(double) * (size_t)nsk * ns);
  if (c.hxc) {
    const size_t nc = hxc_spectrum_elems(c);
    b.take(c.d_Vloc, sizeof(double) * c.nd);
    b.take(c.d_rho_in, sizeof(double) * c.nd);
    b.take(c.d_hx, sizeof(double) * c.nd * kHxcWindow);
    b.take(c.d_hf, sizeof(double) * c.nd * kHxcWindow);
    b.take(c.d_hbar, sizeof(double) * c.nd * 2);
    b.take(c.d_hspec, sizeof(double) * nc * 4);
    b.take(c.d_hsym, sizeof(double) * (c.p.n[0] / 2 + 1 + c.p.n[1] + c.p.n[2]));
    b.take(c.d_hpart, sizeof(double) * hxc_partial_elems());
  }
  // ---- position dependent
  b.take(c.d_supp, sizeof(int) * c.supp.size());
  b.take(c.d_boff, sizeof(int64_t) * c.boff.size());
  b.take(c.d_bnj, sizeof(int) * c.bnj.size());
  b.take(c.d_bj, sizeof(int) * c.bj.size());
  b.take(c.d_bsrc, sizeof(int64_t) * c.bsrc.size());
  b.take(c.d_pboff, sizeof(int64_t) * c.pboff.size());
  b.take(c.d_pbnj, sizeof(int) * c.pbnj.size());
  b.take(c.d_pbsrc, sizeof(int64_t) * c.pbsrc.size());
  b.take(c.d_pdest, sizeof(int64_t) * c.pdest.size());
  b.take(c.d_jrow, sizeof(int64_t) * c.jrow.size());
  std::vector<void*> cscv(c.p.nk), bval(c.p.nk), pbval(c.p.nk);
  for (int k = 0; k < c.p.nk; ++k) {
    b.take(pbval[k], es * c.pbsrc.size());
    b.take(cscv[k], es * c.nval);
    b.take(bval[k], es * c.bsrc.size());
  }
  if (assign) { c.d_cscv = cscv; c.d_bval = bval; c.d_pbval = pbval; }
  std::vector<void*> pp(nsk, nullptr);
  b.take(pp[0], es * project_partial_elems(c));
  for (int i = 1; i < nsk; ++i) b.take(pp[i], es * project_partial_elems(c));
  if (assign) { c.d_ppart = pp[0]; c.d_ppart_sk = pp; }
  b.take(c.d_momcsc, es * (size_t)c.nval);
  for (int d = 0; d < 3; ++d) b.take(c.d_mom[d], es * c.pbsrc.size());
  return b.off;
}

hcu_status upload_structure(Ctx& c);
void aimd_coefficients(const Ctx& c, double* out);

hcu_status check_ctx(const hcu_ctx* ctx) {
  if (!ctx) return HCU_INVALID_ARG;
  if (!ctx->bound) { const_cast<hcu_ctx*>(ctx)->err = "context not bound to device memory"; return HCU_NOT_BOUND; }
  return HCU_OK;
}

hcu_status fail(Ctx& c, hcu_status s, const std::string& msg) {
  c.err = msg;
  return s;
}

// coupling matrices of every block for one spin: diag(gamma) for KB, U(1/2 - D_in) for Hubbard
hcu_status upload_coupling(Ctx& c) {
  const int nh = (int)c.hub_atoms.size();
  for (int s = 0; s < c.p.nspin; ++s) {
    std::vector<double> cp(std::max(c.coup_size, 1), 0.0);
    for (const BlockDesc& b : c.blocks) {
      double* M = cp.data() + b.coup_off;
      if (b.type == 0) {
        int m0 = 0;
        for (int ch = 0; ch < b.nchan; ++ch) {
          const int nmc = 2 * b.chan_l[ch] + 1;
          for (int m = 0; m < nmc; ++m) M[(m0 + m) * b.nm + m0 + m] = b.chan_gamma[ch];
          m0 += nmc;
        }
      } else {
        const double U = c.hub_U[b.hub];
        const double* D = c.D_in.data() + ((size_t)s * nh + b.hub) * 25;
        for (int i = 0; i < b.nm; ++i)
          for (int j = 0; j < b.nm; ++j) M[i * b.nm + j] = U * ((i == j ? 0.5 : 0.0) - D[i * 5 + j]);
      }
    }
    HCU_HIP(hipMemcpyAsync(c.d_coup[s], cp.data(), sizeof(double) * c.coup_size, hipMemcpyHostToDevice, c.stream));
    HCU_HIP(hipStreamSynchronize(c.stream));   // cp is released at the end of this iteration
  }
  return HCU_OK;
}

// Symmetric tridiagonal eigenvalues (small, host): cyclic Jacobi on the dense
// matrix.
void small_sym_eigvals(std::vector<double> A, int n, std::vector<double>& ev) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
    if (off < 1e-30) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double th = (A[q * n + q] - A[p * n + p]) / (2 * apq);
        double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1));
        double cs = 1 / std::sqrt(t * t + 1), sn = t * cs;
        for (int r = 0; r < n; ++r) {
          double arp = A[r * n + p], arq = A[r * n + q];
          A[r * n + p] = cs * arp - sn * arq;
          A[r * n + q] = sn * arp + cs * arq;
        }
        for (int r = 0; r < n; ++r) {
          double apr = A[p * n + r], aqr = A[q * n + r];
          A[p * n + r] = cs * apr - sn * aqr;
          A[q * n + r] = sn * apr + cs * aqr;
        }
      }
  }
  ev.resize(n);
  for (int i = 0; i < n; ++i) ev[i] = A[i * n + i];
  std::sort(ev.begin(), ev.end());
}

// Hs C = S C diag(lam), C^H S C = I (FP64 on the device): Cholesky S = U^H U,
// A = U^-H Hs U^-1, A = Q diag(lam) Q^H, C = U^-1 Q.  Overwrites d_S with U
// and d_Hs with C.  Sets d_info (nonzero: S not positive definite or the
// tridiagonal eigensolver did not converge).
hcu_status generalized_eig(Ctx& c, int n, bool cp, double* lam) {
  rocblas_status r;
  launch_rr_guard_in(c.d_S, c.d_Hs, n, cp ? 2 : 1, c.d_info, c.stream);
  if (cp) {
    auto* S = (rocblas_double_complex*)c.d_S;
    auto* A = (rocblas_double_complex*)c.d_Hs;
    const rocblas_double_complex one{1.0, 0.0};
    r = rocsolver_zpotrf(c.blas, rocblas_fill_upper, n, S, n, c.d_info);
    if (r == rocblas_status_success) launch_rr_guard_chol(c.d_S, c.d_Hs, n, 2, c.d_info, c.stream);
    if (r == rocblas_status_success)
      r = rocblas_ztrsm(c.blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_conjugate_transpose,
                        rocblas_diagonal_non_unit, n, n, &one, S, n, A, n);
    if (r == rocblas_status_success)
      r = rocblas_ztrsm(c.blas, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                        rocblas_diagonal_non_unit, n, n, &one, S, n, A, n);
    if (hetrd_small_ok(n) && c.part_elems >= 2 * (size_t)n * n) {
      // tridiagonal form in one workgroup (eig.hip), then the library's
      // divide and conquer into a complex eigenvector matrix (the Gram
      // partials) and the back-transformation by the reflectors
      auto* Z = (rocblas_double_complex*)c.d_part;
      double* e = c.d_E;
      auto* tau = (rocblas_double_complex*)(c.d_E + n);
      if (r == rocblas_status_success)
        launch_hetrd_small((cplx<double>*)c.d_Hs, n, n, lam, e, (cplx<double>*)tau, c.stream);
      if (r == rocblas_status_success)
        r = rocsolver_zstedc(c.blas, rocblas_evect_tridiagonal, n, lam, e, Z, n, c.d_info + 1);
      if (r == rocblas_status_success)
        r = rocsolver_zunmtr(c.blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none, n, n, A, n, tau,
                             Z, n);
      if (r == rocblas_status_success)
        r = rocblas_ztrsm(c.blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none,
                          rocblas_diagonal_non_unit, n, n, &one, S, n, Z, n);
      if (r == rocblas_status_success &&
          hipMemcpyAsync(A, Z, 2 * sizeof(double) * n * n, hipMemcpyDeviceToDevice, c.stream) != hipSuccess)
        r = rocblas_status_internal_error;
    } else {
      if (r == rocblas_status_success)
        r = rocsolver_zheevd(c.blas, rocblas_evect_original, rocblas_fill_upper, n, A, n, lam, c.d_E, c.d_info + 1);
      if (r == rocblas_status_success)
        r = rocblas_ztrsm(c.blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none,
                          rocblas_diagonal_non_unit, n, n, &one, S, n, A, n);
    }
  } else {
    const double one = 1.0;
    r = rocsolver_dpotrf(c.blas, rocblas_fill_upper, n, c.d_S, n, c.d_info);
    if (r == rocblas_status_success) launch_rr_guard_chol(c.d_S, c.d_Hs, n, 1, c.d_info, c.stream);
    if (r == rocblas_status_success)
      r = rocblas_dtrsm(c.blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_transpose,
                        rocblas_diagonal_non_unit, n, n, &one, c.d_S, n, c.d_Hs, n);
    if (r == rocblas_status_success)
      r = rocblas_dtrsm(c.blas, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                        rocblas_diagonal_non_unit, n, n, &one, c.d_S, n, c.d_Hs, n);
    if (sytrd_small_ok(n) && c.part_elems >= (size_t)n * n) {
      // tridiagonal form in one workgroup (eig.hip), then the library's
      // tridiagonal divide and conquer and back-transformation; the
      // eigenvectors are formed in the Gram partials (free after the Gram
      // reduction), the tridiagonal in d_E (off-diagonal, then tau)
      double* Z = c.d_part;
      double* e = c.d_E;
      double* tau = c.d_E + n;
      if (r == rocblas_status_success) launch_sytrd_small(c.d_Hs, n, n, lam, e, tau, c.stream);
      if (r == rocblas_status_success)
        r = rocsolver_dstedc(c.blas, rocblas_evect_tridiagonal, n, lam, e, Z, n, c.d_info + 1);
      if (r == rocblas_status_success)
        r = rocsolver_dormtr(c.blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none, n, n, c.d_Hs, n,
                             tau, Z, n);
      if (r == rocblas_status_success)
        r = rocblas_dtrsm(c.blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none,
                          rocblas_diagonal_non_unit, n, n, &one, c.d_S, n, Z, n);
      if (r == rocblas_status_success &&
          hipMemcpyAsync(c.d_Hs, Z, sizeof(double) * n * n, hipMemcpyDeviceToDevice, c.stream) != hipSuccess)
        r = rocblas_status_internal_error;
    } else {
      if (r == rocblas_status_success)
        r = rocsolver_dsyevd(c.blas, rocblas_evect_original, rocblas_fill_upper, n, c.d_Hs, n, lam, c.d_E,
                             c.d_info + 1);
      if (r == rocblas_status_success)
        r = rocblas_dtrsm(c.blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_none,
                          rocblas_diagonal_non_unit, n, n, &one, c.d_S, n, c.d_Hs, n);
    }
  }
  if (r != rocblas_status_success) return fail(c, HCU_DEVICE, "rocSOLVER/rocBLAS call failed in the eigensolve");
  return HCU_OK;
}

// ------------------------------------------------------------------ typed steps
// Projection of y onto every atom-centred function: P = Phi^H y dV,
// Q = C P (Q transposed).
template <typename T>
void project_t(Ctx& c, int spin, int ik, const T* y, int64_t ldy, int ncol) {
  ProfScope ps(c, PK_PROJECT);
  const int sk = sk_index(c, spin, ik);
  launch_project_brick<T>(c, ik, y, ncol, ldy, c.d_coup[spin], (T*)c.d_P[sk], (T*)c.d_Q[sk], c.stream);
}

// P and Q of the context's own block X of (spin, ik): the projections the
// last Rayleigh-Ritz rotation left (P(X) = P(Y) C, equal to projecting X up
// to rounding) with the coupling of the current D applied anew, when they
// are current; else projected.
template <typename T>
hcu_status project_x_t(Ctx& c, int spin, int ik, const T* X, int ncol) {
  const int sk = sk_index(c, spin, ik);
  if (c.nproj > 0 && X == (const T*)c.d_X[sk] && ncol == c.p.ns && sk < (int)c.px_valid.size() && c.px_valid[sk]) {
    ProfScope ps(c, PK_PROJECT);
    HCU_HIP(hipMemcpyAsync(c.d_P[sk], c.d_PX[sk], esize(c) * (size_t)ncol * c.nproj, hipMemcpyDeviceToDevice,
                           c.stream));
    launch_couple<T>(c, (const T*)c.d_P[sk], ncol, c.d_coup[spin], (T*)c.d_Q[sk], c.stream);
    return HCU_OK;
  }
  project_t<T>(c, spin, ik, X, c.nd, ncol);
  return HCU_OK;
}

// Y (already holding the local part) += alpha Phi Q.
template <typename T>
void scatter_t(Ctx& c, int spin, int ik, T* Y, int64_t ldy, int ncol, double alpha) {
  ProfScope ps(c, PK_SCATTER);
  launch_nl_scatter<T>(c, ik, Y, ldy, ncol, (const T*)c.d_Q[sk_index(c, spin, ik)], alpha, c.stream);
}

// Y += alpha Phi Q and, in the same pass (real blocks), P and Q of the
// updated Y for the next Chebyshev step.
template <typename T>
void scatter_project_t(Ctx& c, int spin, int ik, T* Y, int64_t ldy, int ncol, double alpha) {
  const int sk = sk_index(c, spin, ik);
  {
    ProfScope ps(c, PK_FUSED);   // the fused kernel alone
    launch_scatter_project<T>(c, ik, Y, ldy, ncol, (const T*)c.d_Q[sk], alpha, c.d_coup[spin], (T*)c.d_P[sk],
                              (T*)c.d_Q[sk], c.stream, 1);
  }
  ProfScope ps(c, PK_SCATTER);   // partial sums and coupling of the projections
  launch_scatter_project<T>(c, ik, Y, ldy, ncol, (const T*)c.d_Q[sk], alpha, c.d_coup[spin], (T*)c.d_P[sk],
                            (T*)c.d_Q[sk], c.stream, 2);
}

// The partial sums and coupling that follow a fused pass run in a batched
// launch, reading block sk's own partials.
template <typename T>
void scatter_project_tail_t(Ctx& c, int spin, int ik, T* Y, int64_t ldy, int ncol, double alpha) {
  const int sk = sk_index(c, spin, ik);
  void* const p0 = c.d_ppart;
  c.d_ppart = c.d_ppart_sk[sk];
  {
    ProfScope ps(c, PK_SCATTER);
    launch_scatter_project<T>(c, ik, Y, ldy, ncol, (const T*)c.d_Q[sk], alpha, c.d_coup[spin], (T*)c.d_P[sk],
                              (T*)c.d_Q[sk], c.stream, 2);
  }
  c.d_ppart = p0;
}

// proj_in = false: P and Q of X are already current (left by the step that
// produced X).
template <typename T>
void apply_h_t(Ctx& c, int spin, int ik, const T* X, int64_t ldx, T* Y, int64_t ldy, int ncol, bool proj_in = true) {
  if (c.nproj > 0 && proj_in) project_t<T>(c, spin, ik, X, ldx, ncol);
  {
    ProfScope ps(c, PK_STENCIL);
    launch_stencil<T>(c, ik, X, ldx, nullptr, 0, Y, ldy, ncol, 1.0, 0.0, 0.0, c.stream);
  }
  if (c.nproj > 0) scatter_t<T>(c, spin, ik, Y, ldy, ncol, 1.0);
}

// One Chebyshev step: out = alpha (H y - c y) - beta yprev.
// proj_in: project y first (else its P and Q are current); proj_out: leave P
// and Q of out behind (fused with the scatter).
template <typename T>
void cheb_step_t(Ctx& c, int spin, int ik, const T* y, int64_t ldy, const T* yprev, int64_t ldp, T* out,
                 int64_t ldo, int ncol, double alpha, double cc, double beta, bool proj_in, bool proj_out) {
  if (c.nproj > 0 && proj_in) project_t<T>(c, spin, ik, y, ldy, ncol);
  {
    ProfScope ps(c, PK_STENCIL);
    launch_stencil<T>(c, ik, y, ldy, yprev, ldp, out, ldo, ncol, alpha, cc, beta, c.stream);
  }
  if (c.nproj > 0) {
    if (proj_out) scatter_project_t<T>(c, spin, ik, out, ldo, ncol, alpha);
    else scatter_t<T>(c, spin, ik, out, ldo, ncol, alpha);
  }
}

// Returns the index of the work block that holds the filtered block.
// project_last: leave P and Q of the filtered block behind (for H Y next).
// Between steps the projections come out of the fused scatter when the
// block type allows it.
// proj_x = false: P and Q of X are already current.
template <typename T>
int filter_t(Ctx& c, int spin, int ik, const T* X, int64_t ldx, int ncol, int m, double a, double b, double aL,
             bool project_last = false, bool proj_x = true) {
  const bool fuse = scatter_project_ok<T>(c);
  const double e = (b - a) / 2, cc = (b + a) / 2;
  double sigma = e / (aL - cc);
  const double tau = 2.0 / sigma;
  const int64_t nd = c.nd;
  void** W = &c.d_W[3 * sk_index(c, spin, ik)];
  cheb_step_t<T>(c, spin, ik, X, ldx, nullptr, 0, (T*)W[0], nd, ncol, sigma / e, cc, 0.0, proj_x,
                 fuse && (m > 1 || project_last));
  const T* prev = X;
  int64_t ldp = ldx;
  int cur = 0;
  for (int i = 2; i <= m; ++i) {
    const double s2 = 1.0 / (tau - sigma);
    const int out = (cur + 1) % 3;
    cheb_step_t<T>(c, spin, ik, (const T*)W[cur], nd, prev, ldp, (T*)W[out], nd, ncol, 2.0 * s2 / e, cc,
                   sigma * s2, !fuse, fuse && (i < m || project_last));
    prev = (const T*)W[cur];
    ldp = nd;
    cur = out;
    sigma = s2;
  }
  return cur;
}

// Queue Rayleigh-Ritz for (spin, k) block sk: S, Hs from Y and H Y, FP64
// generalized eigensolve, X = Y C, projections of X; results read by
// rr_finish after a stream synchronisation.
template <typename T>
hcu_status rr_t(Ctx& c, int sk, T* Y, T* HY) {
  const int ns = c.p.ns;
  const int64_t nd = c.nd;
  T* X = (T*)c.d_X[sk];
  if (c.nproj > 0)
    HCU_HIP(hipMemcpyAsync(c.d_PY[sk], c.d_P[sk], esize(c) * (size_t)ns * c.nproj, hipMemcpyDeviceToDevice,
                           c.stream));
  {
    ProfScope ps(c, PK_GRAM);
    launch_gram2<T>(c, Y, HY, ns, nd, c.d_S, c.d_Hs, c.stream);
  }
  HCU_HIP(hipGetLastError());
  const bool cp = sizeof(T) > sizeof(typename real_of<T>::type);
  {
    ProfScope ps(c, PK_EIG, true);
    hcu_status es = generalized_eig(c, ns, cp, c.d_lam + (size_t)sk * ns);
    if (es != HCU_OK) return es;
  }
  launch_convert_c<T>(c.d_Hs, (T*)c.d_Cb, ns, cp ? 1 : 0, c.stream);
  {
    ProfScope ps(c, PK_ROTATE, true);   // a library call for real blocks
    launch_rotate<T>(c, Y, nd, (const T*)c.d_Cb, X, ns, c.stream);
  }
  if (c.nproj > 0) {
    launch_rotate_proj<T>(c, (const T*)c.d_PY[sk], (const T*)c.d_Cb, (T*)c.d_PX[sk], ns, c.stream);
    if ((int)c.px_valid.size() <= sk) c.px_valid.resize(sk + 1, 0);
    c.px_valid[sk] = 1;   // P(X) = P(Y) C: the next filter starts from it
  }
  HCU_HIP(hipGetLastError());
  HCU_HIP(hipMemcpyAsync(c.h_info + kInfoPerBlock * sk, c.d_info, 3 * sizeof(int), hipMemcpyDeviceToHost, c.stream));
  return HCU_OK;
}

// After the stream has synchronised: check the eigensolve, update bounds.
hcu_status rr_finish(Ctx& c, int sk) {
  const int ns = c.p.ns;
  const int* info2 = c.h_info + kInfoPerBlock * sk;
  if (info2[2] != 0) return fail(c, HCU_NAN, "non-finite entries in the Rayleigh-Ritz matrices");
  if (info2[0] != 0)
    return fail(c, HCU_NOT_SPD, "Gram matrix of the filtered block not positive definite (potrf info=" +
                                    std::to_string(info2[0]) + ")");
  if (info2[1] != 0)
    return fail(c, HCU_DEVICE, "subspace eigensolver did not converge (info=" + std::to_string(info2[1]) + ")");
  std::vector<double> lam(ns);
  hipError_t e = hipMemcpy(lam.data(), c.d_lam + (size_t)sk * ns, sizeof(double) * ns, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(c, HCU_DEVICE, hipGetErrorString(e));
  for (int i = 0; i < ns; ++i)
    if (!std::isfinite(lam[i])) return fail(c, HCU_NAN, "non-finite Ritz value");
  c.bounds[3 * sk] = lam[ns - 1];
  c.bounds[3 * sk + 2] = lam[0];
  prof_resolve(c);
  return HCU_OK;
}

template <typename T>
hcu_status pass_t(Ctx& c, int spin, int ik, double* filter_ms) {
  const int sk = sk_index(c, spin, ik);
  const int ns = c.p.ns;
  const int64_t nd = c.nd;
  T* X = (T*)c.d_X[sk];
  const double a = c.bounds[3 * sk], b = c.bounds[3 * sk + 1], aL = c.bounds[3 * sk + 2];
  hipEvent_t e0, e1;
  HCU_HIP(hipEventCreate(&e0));
  HCU_HIP(hipEventCreate(&e1));
  HCU_HIP(hipEventRecord(e0, c.stream));
  const bool fuse = scatter_project_ok<T>(c);
  // the filter's first projection (of X) before the filter
  if (c.nproj > 0) {
    const hcu_status ps = project_x_t<T>(c, spin, ik, X, ns);
    if (ps != HCU_OK) return ps;
  }
  const int iy = filter_t<T>(c, spin, ik, X, nd, ns, c.p.degree, a, b, aL, fuse, false);
  const int ih = (iy + 1) % 3;
  T* Y = (T*)c.d_W[3 * sk + iy];
  T* HY = (T*)c.d_W[3 * sk + ih];
  apply_h_t<T>(c, spin, ik, Y, nd, HY, nd, ns, !fuse);
  HCU_HIP(hipEventRecord(e1, c.stream));
  hcu_status s = rr_t<T>(c, sk, Y, HY);
  if (s != HCU_OK) return s;
  HCU_HIP(hipStreamSynchronize(c.stream));
  float ms = 0;
  hipEventElapsedTime(&ms, e0, e1);
  if (filter_ms) *filter_ms += ms;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return rr_finish(c, sk);
}

// ------------------------------------------------------------------ batches
struct BProb {
  Ctx* c;
  int spin, ik, sk;
  double e, cc, sigma, tau;
};

// One filter + Rayleigh-Ritz pass on every problem of a batch in lockstep:
// per Chebyshev step the projections and scatters run per problem and the
// stencils of all problems run as persistent launches (one per tile shape).
// The launches of the whole pass are planned first and their job tables
// uploaded once, so the host never waits on the device inside the pass.
// All contexts share the stream and the filter degree.
// Rayleigh-Ritz of every problem of a pass.  The eigensolves are chains of
// small library kernels bound by launch latency, so with several problems
// they run on up to kRRLanes side streams at once: problem i goes to lane
// i % lanes, the j-th problem of a context uses the context's scratch slot
// j % lanes (problems that share a slot also share a lane, so they run in
// order), and the lead stream waits for every lane before it goes on.
struct RRSwap {   // a context's Rayleigh-Ritz scratch, handle and stream redirected to a slot and lane
  Ctx& c;
  hipStream_t st0;
  rocblas_handle blas0;
  double *part0, *S0, *Hs0, *E0;
  void* Cb0;
  int* info0;
  RRSwap(Ctx& c_, int slot, hipStream_t lane)
      : c(c_), st0(c_.stream), blas0(c_.blas), part0(c_.d_part), S0(c_.d_S), Hs0(c_.d_Hs), E0(c_.d_E),
        Cb0(c_.d_Cb), info0(c_.d_info) {
    if (slot > 0) {
      const Ctx::RRSlot& r = c.rr_slots[slot - 1];
      c.blas = r.blas;
      c.d_part = r.part;
      c.d_S = r.S;
      c.d_Hs = r.Hs;
      c.d_E = r.E;
      c.d_Cb = r.Cb;
      c.d_info = r.info;
    }
    c.stream = lane;
    rocblas_set_stream(c.blas, lane);
  }
  ~RRSwap() {
    if (c.blas == blas0) rocblas_set_stream(c.blas, st0);
    c.stream = st0;
    c.blas = blas0;
    c.d_part = part0;
    c.d_S = S0;
    c.d_Hs = Hs0;
    c.d_E = E0;
    c.d_Cb = Cb0;
    c.d_info = info0;
  }
};

// Side streams of a batch (created on first use, owned by the lead context)
// and the event pairs that order them against the lead stream.
hcu_status side_lanes(Ctx& lead, int nl) {
  while ((int)lead.rr_streams.size() < nl) {
    hipStream_t st;
    HCU_HIP_CTX(lead, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    lead.rr_streams.push_back(st);
  }
  while ((int)lead.rr_events.size() < 1 + nl) {
    hipEvent_t e;
    HCU_HIP_CTX(lead, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    lead.rr_events.push_back(e);
  }
  return HCU_OK;
}
// the lanes wait for everything queued on the lead stream so far
hcu_status fan_out(Ctx& lead, int nl) {
  HCU_HIP_CTX(lead, hipEventRecord(lead.rr_events[0], lead.stream));
  for (int l = 0; l < nl; ++l) HCU_HIP_CTX(lead, hipStreamWaitEvent(lead.rr_streams[l], lead.rr_events[0], 0));
  return HCU_OK;
}
// the lead stream waits for everything queued on the lanes so far
hcu_status fan_in(Ctx& lead, int nl) {
  for (int l = 0; l < nl; ++l) {
    HCU_HIP_CTX(lead, hipEventRecord(lead.rr_events[1 + l], lead.rr_streams[l]));
    HCU_HIP_CTX(lead, hipStreamWaitEvent(lead.stream, lead.rr_events[1 + l], 0));
  }
  return HCU_OK;
}

struct StreamSwap {   // a context's kernels queued on another stream for a while
  Ctx& c;
  hipStream_t st0;
  StreamSwap(Ctx& c_, hipStream_t st) : c(c_), st0(c_.stream) {
    if (st) c.stream = st;
  }
  ~StreamSwap() { c.stream = st0; }
};

template <typename T, typename Op>
hcu_status rr_all_t(std::vector<BProb>& probs, Ctx& lead, const std::vector<Op>& ys, const std::vector<Op>& hys) {
  const int np = (int)probs.size();
  const int nl = std::min(np, kRRLanes);
  if (nl <= 1) {
    for (int i = 0; i < np; ++i) {
      hcu_status s = rr_t<T>(*probs[i].c, probs[i].sk, (T*)ys[i].out, (T*)hys[i].out);
      if (s != HCU_OK) return s;
    }
    return HCU_OK;
  }
  hcu_status s = side_lanes(lead, nl);
  if (s != HCU_OK) return s;
  s = fan_out(lead, nl);
  if (s != HCU_OK) return s;
  std::vector<std::pair<const Ctx*, int>> seen;
  for (int i = 0; i < np && s == HCU_OK; ++i) {
    Ctx& c = *probs[i].c;
    int j = 0;
    auto it = std::find_if(seen.begin(), seen.end(), [&](const std::pair<const Ctx*, int>& e) { return e.first == &c; });
    if (it == seen.end()) seen.push_back({&c, 1});
    else j = it->second++;
    const int slot = j % nl;
    if (slot > (int)c.rr_slots.size()) {
      s = fail(c, HCU_INVALID_ARG, "no Rayleigh-Ritz scratch slot for this block");
      break;
    }
    RRSwap sw(c, slot, lead.rr_streams[i % nl]);
    s = rr_t<T>(c, probs[i].sk, (T*)ys[i].out, (T*)hys[i].out);
  }
  // the lead stream waits for every lane, also after a failure
  const hcu_status s2 = fan_in(lead, nl);
  return s != HCU_OK ? s : s2;
}

template <typename T>
hcu_status batch_pass_t(std::vector<BProb>& probs, Ctx& lead, double* filter_ms) {
  hipStream_t st = lead.stream;
  const int np = (int)probs.size();
  const int m = lead.p.degree;
  // ---- plan: per step (1..m filter steps, m+1 = H Y) the jobs of every problem
  for (BProb& q : probs) {
    Ctx& c = *q.c;
    const double a = c.bounds[3 * q.sk], b = c.bounds[3 * q.sk + 1], aL = c.bounds[3 * q.sk + 2];
    q.e = (b - a) / 2;
    q.cc = (b + a) / 2;
    q.sigma = q.e / (aL - q.cc);
    q.tau = 2.0 / q.sigma;
  }
  struct StepOp { const void* in; void* out; double alpha; };   // per (step, problem): scatter target and scale
  std::vector<std::vector<StepOp>> ops(m + 1, std::vector<StepOp>(np));
  std::vector<unsigned char> host;
  std::vector<BatchLaunch> launches;
  std::vector<size_t> first(m + 2, 0);
  std::vector<int> cur(np, 0);
  std::vector<const void*> prev(np);
  std::vector<StencilJob> jobs(np);
  for (int step = 1; step <= m + 1; ++step) {
    for (int i = 0; i < np; ++i) {
      BProb& q = probs[i];
      Ctx& c = *q.c;
      void** W = &c.d_W[3 * q.sk];
      if (step == 1) {
        const void* X = c.d_X[q.sk];
        jobs[i] = StencilJob{&c, q.ik, X, c.nd, nullptr, 0, W[0], c.nd, c.p.ns, q.sigma / q.e, q.cc, 0.0};
        ops[0][i] = StepOp{X, W[0], q.sigma / q.e};
        prev[i] = X;
      } else if (step <= m) {
        const double s2 = 1.0 / (q.tau - q.sigma);
        const double alpha = 2.0 * s2 / q.e, beta = q.sigma * s2;
        const int out = (cur[i] + 1) % 3;
        jobs[i] = StencilJob{&c, q.ik, W[cur[i]], c.nd, prev[i], c.nd, W[out], c.nd, c.p.ns, alpha, q.cc, beta};
        ops[step - 1][i] = StepOp{W[cur[i]], W[out], alpha};
        prev[i] = W[cur[i]];
        cur[i] = out;
        q.sigma = s2;
      } else {
        const int out = (cur[i] + 1) % 3;
        jobs[i] = StencilJob{&c, q.ik, W[cur[i]], c.nd, nullptr, 0, W[out], c.nd, c.p.ns, 1.0, 0.0, 0.0};
        ops[m][i] = StepOp{W[cur[i]], W[out], 1.0};
      }
    }
    first[step - 1] = launches.size();
    hcu_status s = plan_stencil_batch<T>(jobs, host, launches);
    if (s != HCU_OK) return fail(lead, s, "batched stencil plan failed (shapes)");
  }
  first[m + 1] = launches.size();
  // the fused scatter + projection of steps 0 .. m-1 (every step whose output
  // feeds another filter step) as one launch per step over every block of a
  // context with several (spin, k) blocks (whose blocks would otherwise run
  // one after another on one stream): job tables planned here and uploaded
  // with the stencil jobs.  The members of a batch of several contexts keep
  // their own launches on the side streams, which overlap better (measured:
  // 16-cell batch 214 against 250 ms per pass with one launch for all)
  bool fuse_all = true;
  for (int i = 0; i < np; ++i)
    fuse_all &= probs[i].c == probs[0].c && probs[i].c->nproj > 0 && scatter_project_ok<T>(*probs[i].c);
  std::vector<size_t> fjob_off(m, 0);
  std::vector<int> fjob_n(m, 0);
  std::vector<unsigned> fjob_items(m, 0);
  int fNT = 4;
  if (fuse_all) {
    for (int step = 0; step < m; ++step) {
      host.resize((host.size() + 15) & ~size_t(15), 0);
      fjob_off[step] = host.size();
      std::vector<FusedJob> js;
      unsigned items = 0;
      for (int i = 0; i < np; ++i) {
        const BProb& q = probs[i];
        const Ctx& c = *q.c;
        if (c.nproj == 0) continue;
        js.push_back(fused_job_of<T>(c, q.ik, (T*)ops[step][i].out, c.nd, c.p.ns, (const T*)c.d_Q[q.sk],
                                     ops[step][i].alpha, c.d_ppart_sk[q.sk], items));
        items += fused_job_items(c, c.p.ns);
        fNT = std::max(fNT, c.max_ptiles <= 4 ? 4 : 8);
      }
      const size_t at = host.size();
      host.resize(at + js.size() * sizeof(FusedJob));
      if (!js.empty()) std::memcpy(host.data() + at, js.data(), js.size() * sizeof(FusedJob));
      fjob_n[step] = (int)js.size();
      fjob_items[step] = items;
    }
  }
  if (host.size() > kBatchJobBytes) return fail(lead, HCU_OOM, "batched job table too large");
  HCU_HIP_CTX(lead, hipMemcpyAsync(lead.d_jobs, host.data(), host.size(), hipMemcpyHostToDevice, st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (filter_ms) {
    HCU_HIP_CTX(lead, hipEventCreate(&e0));
    HCU_HIP_CTX(lead, hipEventCreate(&e1));
    HCU_HIP_CTX(lead, hipEventRecord(e0, st));
  }
  // ---- execute
  // With several member contexts, each context's projections and scatters
  // go to one side stream (context index mod the lane count; the blocks of
  // one context share its scratch and stay in order on one lane), so that
  // the small members' kernels overlap; the stencil launches stay on the
  // lead stream, ordered against the lanes by events.
  std::vector<int> lane_of(np, 0);
  int nctx = 0;
  {
    std::vector<const Ctx*> seen;
    for (int i = 0; i < np; ++i) {
      auto it = std::find(seen.begin(), seen.end(), probs[i].c);
      if (it == seen.end()) {
        lane_of[i] = (int)seen.size();
        seen.push_back(probs[i].c);
      } else {
        lane_of[i] = (int)(it - seen.begin());
      }
    }
    nctx = (int)seen.size();
  }
  const int nl = std::min(nctx, kRRLanes);
  if (nl > 1) {
    hcu_status s = side_lanes(lead, nl);
    if (s != HCU_OK) return s;
  }
  auto lane_stream = [&](int i) -> hipStream_t { return nl > 1 ? lead.rr_streams[lane_of[i] % nl] : nullptr; };
  for (int step = 0; step <= m; ++step) {
    bool any_proj = false;
    for (int i = 0; i < np; ++i)
      any_proj |= probs[i].c->nproj > 0 && (step == 0 || !scatter_project_ok<T>(*probs[i].c));
    if (any_proj) {
      if (nl > 1 && fan_out(lead, nl) != HCU_OK) return HCU_DEVICE;
      for (int i = 0; i < np; ++i) {
        BProb& q = probs[i];
        if (q.c->nproj > 0 && (step == 0 || !scatter_project_ok<T>(*q.c))) {
          StreamSwap sw(*q.c, lane_stream(i));
          if (step == 0) {
            const hcu_status ps = project_x_t<T>(*q.c, q.spin, q.ik, (const T*)ops[step][i].in, q.c->p.ns);
            if (ps != HCU_OK) return ps;
          } else {
            project_t<T>(*q.c, q.spin, q.ik, (const T*)ops[step][i].in, q.c->nd, q.c->p.ns);
          }
        }
      }
      if (nl > 1 && fan_in(lead, nl) != HCU_OK) return HCU_DEVICE;
    }
    for (size_t l = first[step]; l < first[step + 1]; ++l) {
      ProfScope ps(lead, PK_STENCIL);
      // small launches (a few thousand items) run one workgroup per item: a
      // persistent grid costs more to start and drain than it balances
      const bool persistent = launches[l].total >= kPersistentMinItems;
      hcu_status s = run_stencil_batch<T>(launches[l], lead.d_jobs, persistent ? lead.d_counters : nullptr, st);
      if (s != HCU_OK) return fail(lead, s, "batched stencil launch failed");
    }
    const bool batched_fused = fuse_all && step < m && fjob_n[step] > 0;
    if (batched_fused) {
      ProfScope ps(lead, PK_FUSED);
      launch_scatter_project_batch<T>(reinterpret_cast<const FusedJob*>((const char*)lead.d_jobs + fjob_off[step]),
                                      fjob_n[step], fjob_items[step], lead.pgroup, fNT, st);
    }
    if (nl > 1 && fan_out(lead, nl) != HCU_OK) return HCU_DEVICE;
    for (int i = 0; i < np; ++i) {
      BProb& q = probs[i];
      if (q.c->nproj > 0) {
        StreamSwap sw(*q.c, lane_stream(i));
        // steps before the last leave the projections of their output (the
        // next step's input) behind
        if (batched_fused)
          scatter_project_tail_t<T>(*q.c, q.spin, q.ik, (T*)ops[step][i].out, q.c->nd, q.c->p.ns,
                                    ops[step][i].alpha);
        else if (step < m && scatter_project_ok<T>(*q.c))
          scatter_project_t<T>(*q.c, q.spin, q.ik, (T*)ops[step][i].out, q.c->nd, q.c->p.ns, ops[step][i].alpha);
        else
          scatter_t<T>(*q.c, q.spin, q.ik, (T*)ops[step][i].out, q.c->nd, q.c->p.ns, ops[step][i].alpha);
      }
    }
    if (nl > 1 && fan_in(lead, nl) != HCU_OK) return HCU_DEVICE;
    if (step == m - 1 && filter_ms) HCU_HIP_CTX(lead, hipEventRecord(e1, st));
  }
  // ---- Rayleigh-Ritz per problem: Y = the last filter output, H Y = the last output
  hcu_status s = rr_all_t<T>(probs, lead, ops[m - 1], ops[m]);
  if (s != HCU_OK) return s;
  HCU_HIP_CTX(lead, hipStreamSynchronize(st));
  if (filter_ms) {
    float ms = 0;
    hipEventElapsedTime(&ms, e0, e1);
    *filter_ms += ms;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
  }
  for (BProb& q : probs) {
    hcu_status s = rr_finish(*q.c, q.sk);
    if (s != HCU_OK) return s;
  }
  return HCU_OK;
}

template <typename T>
hcu_status lanczos_t(Ctx& c, int spin, int ik, int steps, double* th_min, double* upper) {
  const int sk = sk_index(c, spin, ik);
  const int64_t nd = c.nd;
  T* v = (T*)c.d_vec;
  T* w = v + nd;
  T* vp = w + nd;
  double* dres = c.d_scal + 8;
  double hres[2];
  auto dot = [&](const T* x, const T* y) -> double {
    launch_dot<T>(c, x, y, nd, dres, c.stream);
    hipMemcpyAsync(hres, dres, 2 * sizeof(double), hipMemcpyDeviceToHost, c.stream);
    hipStreamSynchronize(c.stream);
    return hres[0];
  };
  HCU_HIP(hipMemcpyAsync(v, c.d_v0[sk], esize(c) * nd, hipMemcpyDeviceToDevice, c.stream));
  double nrm = std::sqrt(dot(v, v));
  if (!(nrm > 0)) return fail(c, HCU_INVALID_ARG, "Lanczos start vector is zero");
  launch_scale_copy<T>(v, v, 1.0 / nrm, nd, c.stream);
  HCU_HIP(hipMemsetAsync(vp, 0, esize(c) * nd, c.stream));
  std::vector<double> al, be;
  double bprev = 0;
  for (int j = 0; j < steps; ++j) {
    apply_h_t<T>(c, spin, ik, v, nd, w, nd, 1);
    const double alpha = dot(v, w);
    launch_axpby<T>(c, w, v, -alpha, 0.0, 1.0, nd, c.stream);
    if (j > 0) launch_axpby<T>(c, w, vp, -bprev, 0.0, 1.0, nd, c.stream);
    const double beta = std::sqrt(dot(w, w));
    al.push_back(alpha);
    be.push_back(beta);
    if (beta == 0.0) break;
    HCU_HIP(hipMemcpyAsync(vp, v, esize(c) * nd, hipMemcpyDeviceToDevice, c.stream));
    launch_scale_copy<T>(v, w, 1.0 / beta, nd, c.stream);
    bprev = beta;
  }
  HCU_HIP(hipStreamSynchronize(c.stream));
  const int n = (int)al.size();
  std::vector<double> Tm(n * n, 0.0), ev;
  for (int i = 0; i < n; ++i) {
    Tm[i * n + i] = al[i];
    if (i + 1 < n) Tm[i * n + i + 1] = Tm[(i + 1) * n + i] = be[i];
  }
  small_sym_eigvals(Tm, n, ev);
  const double tmin = ev.front(), bnd = ev.back() + std::fabs(be.back());
  if (!std::isfinite(tmin) || !std::isfinite(bnd)) return fail(c, HCU_NAN, "non-finite Lanczos bound");
  c.bounds[3 * sk] = tmin + (bnd - tmin) / 10.0;
  c.bounds[3 * sk + 1] = bnd;
  c.bounds[3 * sk + 2] = tmin;
  if (th_min) *th_min = tmin;
  if (upper) *upper = bnd;
  return HCU_OK;
}

hcu_status check_kset(Ctx& c) {
  if (c.kset_closed) return HCU_OK;
  return fail(c, HCU_INVALID_ARG,
              "occupation matrices need a k-point set closed under k -> -k with equal weights (D is real only "
              "then); the operator and filter calls accept any k");
}

template <typename T>
hcu_status density_t(Ctx& c, double* rho);

template <typename T>
hcu_status occupations_t(Ctx& c) {
  if (check_kset(c) != HCU_OK) return HCU_INVALID_ARG;
  const int nsk = c.p.nspin * c.p.nk;
  const int nh = (int)c.hub_atoms.size();
  std::vector<double> aux(nsk + nh + c.p.nspin);
  for (int s = 0; s < c.p.nspin; ++s)
    for (int k = 0; k < c.p.nk; ++k) aux[s * c.p.nk + k] = c.kw[k];
  for (int h = 0; h < nh; ++h) aux[nsk + h] = c.hub_U[h];
  for (int s = 0; s < c.p.nspin; ++s) {
    double* p = c.d_coup[s];
    std::memcpy(&aux[nsk + nh + s], &p, sizeof(double*));
  }
  HCU_HIP(hipMemcpyAsync(c.d_scal + 64, aux.data(), sizeof(double) * aux.size(), hipMemcpyHostToDevice, c.stream));
  launch_fermi(c, c.stream);
  for (int s = 0; s < c.p.nspin; ++s)
    for (int k = 0; k < c.p.nk; ++k) launch_occupation_matrix<T>(c, s, k, (const T*)c.d_PX[sk_index(c, s, k)], c.stream);
  launch_energies(c, nullptr, c.stream);
  HCU_HIP(hipGetLastError());
  c.lam.resize((size_t)nsk * c.p.ns);
  c.occ.resize(c.lam.size());
  c.D_out.assign((size_t)c.p.nspin * nh * 25, 0.0);
  double sc[8];
  HCU_HIP(hipMemcpyAsync(c.lam.data(), c.d_lam, sizeof(double) * c.lam.size(), hipMemcpyDeviceToHost, c.stream));
  HCU_HIP(hipMemcpyAsync(c.occ.data(), c.d_occ, sizeof(double) * c.occ.size(), hipMemcpyDeviceToHost, c.stream));
  if (nh > 0)
    HCU_HIP(hipMemcpyAsync(c.D_out.data(), c.d_D, sizeof(double) * c.D_out.size(), hipMemcpyDeviceToHost, c.stream));
  HCU_HIP(hipMemcpyAsync(sc, c.d_scal, sizeof(sc), hipMemcpyDeviceToHost, c.stream));
  HCU_HIP(hipStreamSynchronize(c.stream));
  c.en.mu = sc[0];
  c.en.e_band = sc[1];
  c.en.dc = sc[2];
  c.en.E_U = sc[3];
  c.en.ts = sc[4];
  c.en.F = sc[5];
  c.en.E_H = c.en.E_x = c.en.e_hxc = 0.0;
  if (c.hxc) {
    hcu_status s;
    {
      ProfScope ps(c, PK_HXC, true);
      s = density_t<T>(c, nullptr);
      if (s == HCU_OK) s = hxc_energies(c);
    }
    if (s != HCU_OK) return s;
    c.en.F += c.en.e_hxc;
  }
  c.have_results = true;
  if (!std::isfinite(c.en.F)) return fail(c, HCU_NAN, "non-finite free energy");
  return HCU_OK;
}

template <typename T>
hcu_status density_t(Ctx& c, double* rho) {
  HCU_HIP(hipMemsetAsync(c.d_rho, 0, sizeof(double) * c.p.nspin * c.nd, c.stream));
  const double g = c.p.nspin == 1 ? 2.0 : 1.0;
  for (int s = 0; s < c.p.nspin; ++s)
    for (int k = 0; k < c.p.nk; ++k) {
      const int sk = sk_index(c, s, k);
      launch_density<T>(c, (const T*)c.d_X[sk], c.nd, c.d_occ + (size_t)sk * c.p.ns, g * c.kw[k],
                        c.d_rho + (size_t)s * c.nd, c.stream);
    }
  if (rho)
    HCU_HIP(hipMemcpyAsync(rho, c.d_rho, sizeof(double) * c.p.nspin * c.nd, hipMemcpyDeviceToHost, c.stream));
  HCU_HIP(hipStreamSynchronize(c.stream));
  return HCU_OK;
}

#define DISPATCH(c, FN, ...)                                                          \
  ((c).any_complex ? ((c).mixed ? FN<cplx<float>>(__VA_ARGS__) : FN<cplx<double>>(__VA_ARGS__)) \
                   : ((c).mixed ? FN<float>(__VA_ARGS__) : FN<double>(__VA_ARGS__)))

// Pulay (Anderson) mixing on the upper triangles of D (Sec. II.B mixing).
struct Pulay {
  int h;
  double beta;
  std::vector<std::vector<double>>& xs;
  std::vector<std::vector<double>>& fs;
  std::vector<double> step(const std::vector<double>& x, const std::vector<double>& f) {
    xs.push_back(x);
    fs.push_back(f);
    if ((int)xs.size() > h + 1) { xs.erase(xs.begin()); fs.erase(fs.begin()); }
    const size_t n = x.size();
    std::vector<double> out(n);
    if (xs.size() == 1) {
      for (size_t i = 0; i < n; ++i) out[i] = x[i] + beta * f[i];
      return out;
    }
    const int m = (int)xs.size() - 1;
    // least squares min |f - dF g| via modified Gram-Schmidt QR of dF (n x m)
    std::vector<std::vector<double>> dF(m, std::vector<double>(n)), dX(m, std::vector<double>(n));
    for (int j = 0; j < m; ++j)
      for (size_t i = 0; i < n; ++i) { dF[j][i] = fs[j + 1][i] - fs[j][i]; dX[j][i] = xs[j + 1][i] - xs[j][i]; }
    std::vector<std::vector<double>> Qm = dF;
    std::vector<double> Rm(m * m, 0.0);
    std::vector<int> keep(m, 1);
    for (int j = 0; j < m; ++j) {
      for (int k = 0; k < j; ++k) {
        if (!keep[k]) continue;
        double d = 0;
        for (size_t i = 0; i < n; ++i) d += Qm[k][i] * Qm[j][i];
        Rm[k * m + j] = d;
        for (size_t i = 0; i < n; ++i) Qm[j][i] -= d * Qm[k][i];
      }
      double nr = 0, n0 = 0;
      for (size_t i = 0; i < n; ++i) { nr += Qm[j][i] * Qm[j][i]; n0 += dF[j][i] * dF[j][i]; }
      nr = std::sqrt(nr);
      if (nr <= 1e-12 * std::sqrt(n0) || nr == 0.0) { keep[j] = 0; continue; }
      Rm[j * m + j] = nr;
      for (size_t i = 0; i < n; ++i) Qm[j][i] /= nr;
    }
    std::vector<double> g(m, 0.0), rhs(m, 0.0);
    for (int j = 0; j < m; ++j) {
      if (!keep[j]) continue;
      double d = 0;
      for (size_t i = 0; i < n; ++i) d += Qm[j][i] * f[i];
      rhs[j] = d;
    }
    for (int j = m - 1; j >= 0; --j) {
      if (!keep[j]) continue;
      double v = rhs[j];
      for (int k = j + 1; k < m; ++k) if (keep[k]) v -= Rm[j * m + k] * g[k];
      g[j] = v / Rm[j * m + j];
    }
    for (size_t i = 0; i < n; ++i) {
      double xb = x[i], fb = f[i];
      for (int j = 0; j < m; ++j) { xb -= dX[j][i] * g[j]; fb -= dF[j][i] * g[j]; }
      out[i] = xb + beta * fb;
    }
    return out;
  }
  // The same update with coefficients g fitted elsewhere (the density's,
  // with the density-dependent Hamiltonian): g[j] multiplies the j-th
  // difference of consecutive window entries, oldest first.
  std::vector<double> step_with(const std::vector<double>& x, const std::vector<double>& f,
                                const std::vector<double>& g) {
    xs.push_back(x);
    fs.push_back(f);
    if ((int)xs.size() > h + 1) { xs.erase(xs.begin()); fs.erase(fs.begin()); }
    const int m = (int)xs.size() - 1;
    std::vector<double> out(x.size());
    for (size_t i = 0; i < x.size(); ++i) {
      double xb = x[i], fb = f[i];
      for (int j = 0; j < m && j < (int)g.size(); ++j) {
        xb -= (xs[j + 1][i] - xs[j][i]) * g[j];
        fb -= (fs[j + 1][i] - fs[j][i]) * g[j];
      }
      out[i] = xb + beta * fb;
    }
    return out;
  }
};

std::vector<double> d_to_vec(const Ctx& c, const std::vector<double>& D) {
  std::vector<double> v;
  const int nh = (int)c.hub_atoms.size();
  for (int s = 0; s < c.p.nspin; ++s)
    for (int h = 0; h < nh; ++h) {
      const int nm = 2 * c.hub_l[h] + 1;
      const double* d = D.data() + ((size_t)s * nh + h) * 25;
      for (int i = 0; i < nm; ++i)
        for (int j = i; j < nm; ++j) v.push_back(d[i * 5 + j]);
    }
  return v;
}

void vec_to_d(const Ctx& c, const std::vector<double>& v, std::vector<double>& D) {
  const int nh = (int)c.hub_atoms.size();
  size_t pos = 0;
  for (int s = 0; s < c.p.nspin; ++s)
    for (int h = 0; h < nh; ++h) {
      const int nm = 2 * c.hub_l[h] + 1;
      double* d = D.data() + ((size_t)s * nh + h) * 25;
      for (int i = 0; i < nm; ++i)
        for (int j = i; j < nm; ++j) { d[i * 5 + j] = v[pos]; d[j * 5 + i] = v[pos]; ++pos; }
    }
}


template <typename T>
hcu_status apply_h_v(Ctx& c, int spin, int ik, const void* X, void* Y, int ncol, int64_t ld) {
  apply_h_t<T>(c, spin, ik, (const T*)X, ld, (T*)Y, ld, ncol);
  HCU_HIP(hipGetLastError());
  return HCU_OK;
}

template <typename T>
hcu_status filter_v(Ctx& c, int spin, int ik, const void* X, void* Y, int ncol, int64_t ld, int m, double a,
                    double b, double aL) {
  const int w = filter_t<T>(c, spin, ik, (const T*)X, ld, ncol, m, a, b, aL);
  HCU_HIP(hipMemcpy2DAsync(Y, sizeof(T) * ld, c.d_W[3 * sk_index(c, spin, ik) + w], sizeof(T) * c.nd,
                           sizeof(T) * c.nd, ncol,
                           hipMemcpyDeviceToDevice, c.stream));
  HCU_HIP(hipGetLastError());
  return HCU_OK;
}

template <typename T>
hcu_status gram_v(Ctx& c, const void* Y, const void* HY, int ncol, int64_t ld, double* S, double* Hs) {
  launch_gram2<T>(c, (const T*)Y, (const T*)HY, ncol, ld, c.d_S, c.d_Hs, c.stream);
  HCU_HIP(hipGetLastError());
  const size_t nb = sizeof(double) * (size_t)ncol * ncol * (c.any_complex ? 2 : 1);
  HCU_HIP(hipMemcpyAsync(S, c.d_S, nb, hipMemcpyDeviceToHost, c.stream));
  HCU_HIP(hipMemcpyAsync(Hs, c.d_Hs, nb, hipMemcpyDeviceToHost, c.stream));
  HCU_HIP(hipStreamSynchronize(c.stream));
  return HCU_OK;
}

template <typename T>
hcu_status rotate_v(Ctx& c, const void* Y, const double* C, void* X, int ncol, int64_t ld) {
  const size_t nb = sizeof(double) * (size_t)ncol * ncol * (c.any_complex ? 2 : 1);
  HCU_HIP(hipMemcpyAsync(c.d_C, C, nb, hipMemcpyHostToDevice, c.stream));
  launch_convert_c<T>(c.d_C, (T*)c.d_Cb, ncol, c.any_complex ? 1 : 0, c.stream);
  launch_rotate<T>(c, (const T*)Y, ld, (const T*)c.d_Cb, (T*)X, ncol, c.stream);
  HCU_HIP(hipGetLastError());
  HCU_HIP(hipStreamSynchronize(c.stream));
  return HCU_OK;
}

// Time every admissible stencil tile shape on the full block of (spin 0,
// k 0) and keep the fastest (hcu_autotune).
template <typename T>
hcu_status autotune_t(Ctx& c, hcu_tuning* best) {
  const int n1 = c.p.n[0], n3 = c.p.n[2];
  const int ns = c.p.ns;
  const T* X = (const T*)c.d_X[0];
  const T* Yp = (const T*)c.d_W[1];
  T* Y = (T*)c.d_W[0];   // (spin 0, k 0) work blocks
  std::vector<hcu_tuning> cands;
  const int txs[3] = {n1 <= 128 ? n1 : 64, 64, 32};
  for (int RY : {4, 2, 1})
    for (int ti = 0; ti < 3; ++ti) {
      const int TX = txs[ti];
      if (TX > n1 || (ti > 0 && TX == txs[0])) continue;
      for (int TYt : {1, 2, 3, 4, 6, 8, 9, 12, 14, 16}) {
        if (TX * TYt > 1024 || TX * TYt < 64) continue;
        for (int zd : {1, 2, 4}) {
          const int tz = (n3 + zd - 1) / zd;
          if (zd > 1 && tz < 8) continue;
          for (int ring : {0, 1}) {
            if (!stencil_shape_ok(c, TX, TYt, RY, tz, ring)) continue;
            cands.push_back(hcu_tuning{TX, TYt, RY, tz, ring, 0.0});
          }
        }
      }
    }
  if (cands.empty()) return fail(c, HCU_INVALID_ARG, "no admissible stencil shape");
  hipEvent_t e0, e1;
  HCU_HIP(hipEventCreate(&e0));
  HCU_HIP(hipEventCreate(&e1));
  double best_ms = 1e300;
  hcu_tuning bt = cands[0];
  for (hcu_tuning& t : cands) {
    c.tile_x = t.tile_x; c.tile_yt = t.tile_yt; c.ry = t.ry; c.tile_z = t.tile_z; c.halo_ring = t.halo_ring;
    launch_stencil<T>(c, 0, X, c.nd, Yp, c.nd, Y, c.nd, ns, 0.5, 1.0, 0.25, c.stream);
    // a shape the device cannot launch (e.g. its LDS) is skipped
    if (hipGetLastError() != hipSuccess) { t.stencil_ms = -1.0; continue; }
    HCU_HIP(hipEventRecord(e0, c.stream));
    for (int r = 0; r < 3; ++r) launch_stencil<T>(c, 0, X, c.nd, Yp, c.nd, Y, c.nd, ns, 0.5, 1.0, 0.25, c.stream);
    HCU_HIP(hipGetLastError());
    HCU_HIP(hipEventRecord(e1, c.stream));
    HCU_HIP(hipEventSynchronize(e1));
    float ms = 0;
    hipEventElapsedTime(&ms, e0, e1);
    t.stencil_ms = ms / 3.0;
    if (t.stencil_ms < best_ms) { best_ms = t.stencil_ms; bt = t; }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (best_ms == 1e300) return fail(c, HCU_DEVICE, "no stencil shape could be launched");
  c.tile_x = bt.tile_x; c.tile_yt = bt.tile_yt; c.ry = bt.ry; c.tile_z = bt.tile_z; c.halo_ring = bt.halo_ring;
  if (best) *best = bt;
  return HCU_OK;
}

template <typename T>
hcu_status get_orbitals_v(Ctx& c, int sk, void* dst, int on_device) {
  HCU_HIP(hipMemcpyAsync(dst, c.d_X[sk], sizeof(T) * (size_t)c.nd * c.p.ns,
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c.stream));
  HCU_HIP(hipStreamSynchronize(c.stream));
  return HCU_OK;
}

// Second half of an SCF iteration (after the passes of every (spin, k)):
// occupations, D_out, energies, convergence test, Pulay mixing of D.
hcu_status scf_post(Ctx& c, hcu_scf_step_info* info) {
  const hcu_scf_opts& o = c.scf_opts;
  hcu_status s = DISPATCH(c, occupations_t, c);
  if (s != HCU_OK) return s;
  double res = 0;
  for (size_t i = 0; i < c.D_in.size(); ++i) res += (c.D_out[i] - c.D_in[i]) * (c.D_out[i] - c.D_in[i]);
  res = std::sqrt(res);
  const int natom = std::max(c.p.natom, 1);
  const double dF = c.scf_have_old ? std::fabs(c.en.F - c.scf_F_old) / natom : INFINITY;
  const double res_rho = c.hxc ? c.hxc_res : 0.0;
  if (o.verbose) {
    if (c.hxc)
      std::fprintf(stderr, "[hcu scf] it=%d F=%.12f E_U=%.6e res=%.3e res_rho=%.3e dF=%.3e\n", c.scf_iter, c.en.F,
                   c.en.E_U, res, res_rho, dF);
    else
      std::fprintf(stderr, "[hcu scf] it=%d F=%.12f E_U=%.6e res=%.3e dF=%.3e\n", c.scf_iter, c.en.F, c.en.E_U, res, dF);
  }
  c.scf_F_old = c.en.F;
  c.scf_have_old = true;
  const bool conv = res < o.tol_d && dF < o.tol_f && (!c.hxc || res_rho < o.tol_rho);
  if (info) {
    info->iteration = c.scf_iter;
    info->converged = conv ? 1 : 0;
    info->F = c.en.F;
    info->E_U = c.en.E_U;
    info->residual = res;
    info->dF = dF;
    info->residual_rho = res_rho;
  }
  ++c.scf_iter;
  if (!conv) {
    Pulay mix{o.pulay_history, o.pulay_beta, c.mix_x, c.mix_f};
    std::vector<double> x = d_to_vec(c, c.D_in), xo = d_to_vec(c, c.D_out), f(x.size());
    for (size_t i = 0; i < x.size(); ++i) f[i] = xo[i] - x[i];
    std::vector<double> xn;
    if (c.hxc) {
      // one Pulay step on the density; its coefficients mix D too
      std::vector<double> gamma;
      {
        ProfScope ps(c, PK_HXC, true);
        s = hxc_mix(c, o.pulay_history, o.pulay_beta, o.kerker_k0, gamma);
      }
      if (s != HCU_OK) return s;
      xn = mix.step_with(x, f, gamma);
    } else {
      xn = mix.step(x, f);
    }
    vec_to_d(c, xn, c.D_in);
    s = upload_coupling(c);
    if (s != HCU_OK) return s;
  }
  return HCU_OK;
}

}  // namespace

namespace hcu {
hcu_status compute_density(Ctx& c) { return DISPATCH(c, density_t, c, (double*)nullptr); }

thread_local KTimer* g_ktimer = nullptr;

void prof_resolve(Ctx& c) {
  for (auto& pe : c.ev_pending) {
    float ms = 0;
    if (pe.first >= 0 && hipEventElapsedTime(&ms, pe.second.first, pe.second.second) == hipSuccess) {
      c.prof_ms[pe.first] += ms;
      c.prof_count[pe.first] += 1;
    }
    c.ev_pool.push_back(pe.second.first);
    c.ev_pool.push_back(pe.second.second);
  }
  c.ev_pending.clear();
}
}  // namespace hcu

// ====================================================================== C ABI
extern "C" {

hcu_status hcu_create(const hcu_problem* p, hcu_ctx** out) {
  if (!p || !out) return HCU_INVALID_ARG;
  *out = nullptr;
  hcu_ctx* c = new (std::nothrow) hcu_ctx();
  if (!c) return HCU_OOM;
  auto bad = [&](const char* msg) { c->err = msg; *out = c; return HCU_INVALID_ARG; };
  c->p = *p;
  if (p->n0 < 1 || p->n0 > kMaxR) return bad("n0 must be in 1..6");
  for (int a = 0; a < 3; ++a) {
    if (p->n[a] < 2) return bad("each n_a must be >= 2");
    if (!(p->L[a] > 0)) return bad("cell lengths must be positive");
  }
  if ((int64_t)p->n[0] * p->n[1] * p->n[2] > (int64_t)65535 * 64)
    return bad("grid too large (at most 4194240 points)");
  if (p->nspin != 1 && p->nspin != 2) return bad("nspin must be 1 or 2");
  if (p->nk < 1 || !p->kpts || !p->kw) return bad("need nk >= 1 k-points and weights");
  if (p->natom < 0 || (p->natom > 0 && (!p->atom_species || !p->pos))) return bad("bad atom arrays");
  if (p->nspecies < 0 || (p->nspecies > 0 && !p->species)) return bad("bad species array");
  if (p->ns < 1) return bad("ns must be >= 1");
  if (!(p->kT > 0)) return bad("kT must be positive");
  if (p->degree < 1) return bad("degree must be >= 1");
  if (p->precision != HCU_FP64 && p->precision != HCU_MIXED) return bad("unknown precision");
  if (p->hxc != 0 && p->hxc != 1) return bad("hxc must be 0 or 1");
  if (p->hxc && p->nspin != 1) return bad("the density-dependent Hamiltonian is spin-unpolarised (nspin = 1)");
  const double gs = p->nspin == 1 ? 2.0 : 1.0;
  if (!(p->nelec > 0) || p->nelec >= gs * p->ns * p->nspin) return bad("nelec must be in (0, states available)");
  c->kpts.assign(p->kpts, p->kpts + 3 * p->nk);
  c->kw.assign(p->kw, p->kw + p->nk);
  c->pos.assign(p->pos, p->pos + 3 * p->natom);
  c->atom_species.assign(p->atom_species, p->atom_species + p->natom);
  c->species.assign(p->species, p->species + p->nspecies);
  double wsum = 0;
  for (double w : c->kw) wsum += w;
  if (std::fabs(wsum - 1.0) > 1e-12) return bad("k-point weights must sum to 1");
  for (int a = 0; a < p->natom; ++a)
    if (c->atom_species[a] < 0 || c->atom_species[a] >= p->nspecies) return bad("atom species index out of range");
  for (const hcu_species& s : c->species) {
    if (s.n_kb < 0 || s.n_kb > HCU_MAX_KB) return bad("n_kb out of range");
    for (int ch = 0; ch < s.n_kb; ++ch)
      if (s.kb_l[ch] < 0 || s.kb_l[ch] > 1) return bad("KB channels must have l = 0 or 1");
    if (s.hub_l > 2 || s.hub_l < -1) return bad("hub_l must be -1..2");
    if (!(s.threshold > 0)) return bad("threshold must be positive");
    if (s.n_kb > 0 && !(s.kb_width > 0)) return bad("kb_width must be positive");
    if (s.hub_l >= 0 && !(s.hub_alpha > 0)) return bad("hub_alpha must be positive");
    if (!(s.vloc_width > 0)) return bad("vloc_width must be positive");
  }
  c->nd = p->n[0] * p->n[1] * p->n[2];
  for (int a = 0; a < 3; ++a) c->h[a] = p->L[a] / p->n[a];
  c->dv = c->h[0] * c->h[1] * c->h[2];
  c->mixed = p->precision == HCU_MIXED;
  c->hxc = p->hxc == 1;
  c->any_complex = false;
  for (int k = 0; k < p->nk; ++k)
    if (k_complex(*c, k)) c->any_complex = true;
  // D is stored real; that is exact when every k-point has a partner -k
  // (modulo the reciprocal lattice 2 pi / L_a) of equal weight
  for (int k = 0; k < p->nk && c->kset_closed; ++k) {
    bool found = false;
    for (int q = 0; q < p->nk && !found; ++q) {
      bool same = std::fabs(c->kw[k] - c->kw[q]) <= 1e-12;
      for (int a = 0; a < 3 && same; ++a) {
        const double g = 2.0 * M_PI / p->L[a];
        const double t = (c->kpts[3 * k + a] + c->kpts[3 * q + a]) / g;
        same = std::fabs(t - std::round(t)) <= 1e-9;
      }
      found = same;
    }
    c->kset_closed = found;
  }
  c->p.kpts = nullptr; c->p.kw = nullptr; c->p.pos = nullptr; c->p.atom_species = nullptr; c->p.species = nullptr;
  hcu_status s = build_structure(*c);
  if (s != HCU_OK) { *out = c; return s; }
  for (int nm = 0; nm <= kMaxNm; ++nm) c->nm_count[nm] = 0;
  for (const BlockDesc& b : c->blocks) c->nm_count[b.nm]++;
  int off = 0;
  for (int nm = 0; nm <= kMaxNm; ++nm) { c->nm_offset[nm] = off; off += c->nm_count[nm]; }
  c->D_in.assign((size_t)p->nspin * c->hub_atoms.size() * 25, 0.0);
  c->h_info_store.assign((size_t)kInfoPerBlock * p->nspin * p->nk, 0);
  c->h_info = c->h_info_store.data();
  c->bounds.assign((size_t)3 * p->nspin * p->nk, 0.0);
  c->ws_bytes = layout(*c, nullptr);
  *out = c;
  return HCU_OK;
}

hcu_status hcu_set_profiling(hcu_ctx* ctx, int on) {
  if (!ctx) return HCU_INVALID_ARG;
  if (ctx->bound) { hipStreamSynchronize(ctx->stream); prof_resolve(*ctx); }
  ctx->prof = on != 0;
  for (int i = 0; i < 8; ++i) { ctx->prof_ms[i] = 0; ctx->prof_count[i] = 0; }
  return HCU_OK;
}

hcu_status hcu_get_kernel_times(hcu_ctx* ctx, hcu_kernel_times* t) {
  if (!ctx || !t) return HCU_INVALID_ARG;
  if (ctx->bound) { hipStreamSynchronize(ctx->stream); prof_resolve(*ctx); }
  t->stencil_ms = ctx->prof_ms[PK_STENCIL]; t->stencil_launches = ctx->prof_count[PK_STENCIL];
  t->project_ms = ctx->prof_ms[PK_PROJECT]; t->project_launches = ctx->prof_count[PK_PROJECT];
  t->gram_ms = ctx->prof_ms[PK_GRAM]; t->gram_launches = ctx->prof_count[PK_GRAM];
  t->eig_ms = ctx->prof_ms[PK_EIG]; t->eig_launches = ctx->prof_count[PK_EIG];
  t->hxc_ms = ctx->prof_ms[PK_HXC]; t->hxc_launches = ctx->prof_count[PK_HXC];
  t->rotate_ms = ctx->prof_ms[PK_ROTATE]; t->rotate_launches = ctx->prof_count[PK_ROTATE];
  t->scatter_ms = ctx->prof_ms[PK_SCATTER] + ctx->prof_ms[PK_FUSED];
  t->scatter_launches = ctx->prof_count[PK_SCATTER];
  t->fused_ms = ctx->prof_ms[PK_FUSED]; t->fused_launches = ctx->prof_count[PK_FUSED];
  return HCU_OK;
}

void hcu_destroy(hcu_ctx* ctx) {
  if (!ctx) return;
  for (auto& pe : ctx->ev_pending) { hipEventDestroy(pe.second.first); hipEventDestroy(pe.second.second); }
  for (hipEvent_t e : ctx->ev_pool) hipEventDestroy(e);
  if (ctx->blas) rocblas_destroy_handle(ctx->blas);
  for (Ctx::RRSlot& r : ctx->rr_slots)
    if (r.blas) rocblas_destroy_handle(r.blas);
  for (hipStream_t st : ctx->rr_streams) (void)hipStreamDestroy(st);
  for (hipEvent_t e : ctx->rr_events) (void)hipEventDestroy(e);
  if (ctx->h_info_pinned) (void)hipHostFree(ctx->h_info_pinned);
  hxc_destroy(*ctx);
  delete ctx;
}

const char* hcu_last_error(const hcu_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

hcu_status hcu_workspace_size(const hcu_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return HCU_INVALID_ARG;
  *bytes = ctx->ws_bytes;
  return HCU_OK;
}

int hcu_num_hubbard_atoms(const hcu_ctx* ctx) { return ctx ? (int)ctx->hub_atoms.size() : -1; }

hcu_status hcu_get_sizes(const hcu_ctx* ctx, hcu_sizes* out) {
  if (!ctx || !out) return HCU_INVALID_ARG;
  out->nd = ctx->nd;
  out->nproj = ctx->nproj;
  out->nblocks = (int)ctx->blocks.size();
  out->support_points = (int64_t)ctx->supp.size();
  out->table_nnz = ctx->csr_ptr.empty() ? 0 : ctx->csr_ptr[ctx->nd];
  out->workspace_bytes = ctx->ws_bytes;
  out->max_brick_functions = ctx->pbnj.empty() ? 0 : *std::max_element(ctx->pbnj.begin(), ctx->pbnj.end());
  out->brick_slots = ctx->jrow.empty() ? 0 : ctx->jrow.back();
  return HCU_OK;
}

hcu_status hcu_bind(hcu_ctx* ctx, void* dev_ptr, size_t bytes, void* stream) {
  if (!ctx) return HCU_INVALID_ARG;
  Ctx& c = *ctx;
  if (!dev_ptr) return fail(c, HCU_INVALID_ARG, "null workspace");
  if (((uintptr_t)dev_ptr) % 256) return fail(c, HCU_INVALID_ARG, "workspace must be 256-byte aligned");
  if (bytes < c.ws_bytes) return fail(c, HCU_OOM, "workspace smaller than hcu_workspace_size()");
  c.ws = (char*)dev_ptr;
  c.ws_bound = bytes;
  c.stream = (hipStream_t)stream;
  layout(c, c.ws);
  if (!c.blas) {
    if (rocblas_create_handle(&c.blas) != rocblas_status_success) return fail(c, HCU_DEVICE, "rocblas handle");
  }
  rocblas_set_stream(c.blas, c.stream);
  for (Ctx::RRSlot& r : c.rr_slots)
    if (!r.blas && rocblas_create_handle(&r.blas) != rocblas_status_success)
      return fail(c, HCU_DEVICE, "rocblas handle");
  if (!c.h_info_pinned) {
    HCU_HIP(hipHostMalloc((void**)&c.h_info_pinned, sizeof(int) * c.h_info_store.size(), hipHostMallocDefault));
    std::copy(c.h_info_store.begin(), c.h_info_store.end(), c.h_info_pinned);
    c.h_info = c.h_info_pinned;
  }
  hcu_status s = upload_structure(c);
  if (s != HCU_OK) return s;
  c.bound = true;
  s = upload_coupling(c);
  if (s != HCU_OK) return s;
  HCU_HIP(hipStreamSynchronize(c.stream));
  return HCU_OK;
}

hcu_status hcu_move_atoms(hcu_ctx* ctx, const double* pos, int extrapolate, double* coeffs) {
  hcu_status s = check_ctx(ctx);
  if (s != HCU_OK) return s;
  Ctx& c = *ctx;
  if (!pos) return fail(c, HCU_INVALID_ARG, "null positions");
  for (int i = 0; i < 3 * c.p.natom; ++i)
    if (!std::isfinite(pos[i])) return fail(c, HCU_NAN, "non-finite position");
  // the converged state of the current geometry joins the history
  if (c.have_results) {
    c.aimd_pos.insert(c.aimd_pos.begin(), c.pos);
    c.aimd_D.insert(c.aimd_D.begin(), c.D_out);
    if (c.aimd_pos.size() > 3) { c.aimd_pos.pop_back(); c.aimd_D.pop_back(); }
  }
  const std::vector<double> old = c.pos;
  c.px_valid.clear();   // the projector tables change with the atoms
  c.pos.assign(pos, pos + 3 * c.p.natom);
  s = build_structure(c);
  const size_t need = s == HCU_OK ? layout(c, nullptr, false) : 0;
  if (s != HCU_OK || need > c.ws_bound) {
    c.pos = old;   // the previous geometry stays in force
    const std::string why = s != HCU_OK ? c.err : "the moved atoms need " + std::to_string(need) +
                                                      " workspace bytes, " + std::to_string(c.ws_bound) + " bound";
    build_structure(c);
    return fail(c, s != HCU_OK ? s : HCU_OOM, why);
  }
  c.ws_bytes = need;
  layout(c, c.ws);
  s = upload_structure(c);
  if (s != HCU_OK) return s;
  c.have_results = false;
  c.scf_ready = false;
  double ab[3] = {0.0, 0.0, 0.0};
  if (extrapolate && !c.aimd_D.empty()) {
    aimd_coefficients(c, ab);
    const std::vector<double>& D0 = c.aimd_D[0];
    for (size_t i = 0; i < c.D_in.size(); ++i) {
      double d = D0[i];
      if (c.aimd_D.size() >= 2) d += ab[0] * (D0[i] - c.aimd_D[1][i]);
      if (c.aimd_D.size() >= 3) d += ab[1] * (c.aimd_D[1][i] - c.aimd_D[2][i]);
      c.D_in[i] = d;
    }
  }
  s = upload_coupling(c);
  if (s != HCU_OK) return s;
  if (coeffs) { coeffs[0] = ab[0]; coeffs[1] = ab[1]; coeffs[2] = ab[2]; }
  HCU_HIP(hipStreamSynchronize(c.stream));
  return HCU_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- structure upload and AIMD
namespace {

hcu_status upload_structure(Ctx& c) {
  // per-count block lists and Hubbard block indices
  std::vector<int> lists, hb;
  for (int nm = 0; nm <= kMaxNm; ++nm)
    for (int i = 0; i < (int)c.blocks.size(); ++i)
      if (c.blocks[i].nm == nm) lists.push_back(i);
  for (int i = 0; i < (int)c.blocks.size(); ++i)
    if (c.blocks[i].type == 1) hb.push_back(i);
  if (!lists.empty())
    HCU_HIP(hipMemcpyAsync(c.d_nm_lists, lists.data(), sizeof(int) * lists.size(), hipMemcpyHostToDevice, c.stream));
  if (!hb.empty())
    HCU_HIP(hipMemcpyAsync(c.d_hub_blocks, hb.data(), sizeof(int) * hb.size(), hipMemcpyHostToDevice, c.stream));
  const std::vector<int2> tiles = gram_tiles(c.p.ns, c.any_complex);
  HCU_HIP(hipMemcpyAsync(c.d_tiles, tiles.data(), sizeof(int2) * tiles.size(), hipMemcpyHostToDevice, c.stream));
  hcu_status s = device_tables(c);
  if (s != HCU_OK) return s;
  s = hxc_after_structure(c);   // V_loc + V_H + V_x of the input density
  if (s != HCU_OK) return s;
  HCU_HIP(hipStreamSynchronize(c.stream));   // lists, hb, tiles are released on return
  return HCU_OK;
}

// Coefficients of the second-order extrapolation of an atomic trajectory
// (the scheme the paper adopts for the occupation matrix in AIMD, after the
// charge-density extrapolation it cites, Sec. II.B): with the new positions
// R0 and the recorded ones R1, R2, R3 (most recent first),
//   R0 - R1 ~ a (R1 - R2) + b (R2 - R3)
// in the least-squares sense over all atoms (minimum-norm solution when the
// two history steps are parallel); one recorded step earlier only the first
// term (b = 0).  out = {a, b, order}.
void aimd_coefficients(const Ctx& c, double* out) {
  const size_t nh = c.aimd_pos.size();
  out[0] = out[1] = 0.0;
  out[2] = nh >= 3 ? 2 : nh >= 2 ? 1 : 0;
  if (nh < 2) return;
  const int n = 3 * c.p.natom;
  auto d = [&](const std::vector<double>& a, const std::vector<double>& b, int i) { return a[i] - b[i]; };
  double y1 = 0, s11 = 0;
  double s12 = 0, s22 = 0, y2 = 0;
  for (int i = 0; i < n; ++i) {
    const double r = d(c.pos, c.aimd_pos[0], i);
    const double x1 = d(c.aimd_pos[0], c.aimd_pos[1], i);
    s11 += x1 * x1;
    y1 += x1 * r;
    if (nh >= 3) {
      const double x2 = d(c.aimd_pos[1], c.aimd_pos[2], i);
      s12 += x1 * x2;
      s22 += x2 * x2;
      y2 += x2 * r;
    }
  }
  if (nh < 3) {
    out[0] = s11 > 0 ? y1 / s11 : 0.0;
    return;
  }
  // min-norm solution of [[s11, s12], [s12, s22]] [a, b] = [y1, y2]
  const double tr = s11 + s22, det = s11 * s22 - s12 * s12;
  if (tr <= 0) return;
  if (det > 1e-12 * tr * tr) {
    out[0] = (s22 * y1 - s12 * y2) / det;
    out[1] = (s11 * y2 - s12 * y1) / det;
  } else {
    // rank one: the normal matrix is tr u u^T with u a unit column of it;
    // the minimum-norm least-squares solution is u (u . y) / tr
    double u0 = s11, u1 = s12;
    if (std::fabs(u0) + std::fabs(u1) == 0.0) { u0 = s12; u1 = s22; }
    const double nu = std::sqrt(u0 * u0 + u1 * u1);
    u0 /= nu;
    u1 /= nu;
    const double t = (u0 * y1 + u1 * y2) / tr;
    out[0] = t * u0;
    out[1] = t * u1;
  }
}

}  // namespace

extern "C" {

hcu_status hcu_set_hubbard_occupation(hcu_ctx* ctx, const double* D) {
  if (!ctx) return HCU_INVALID_ARG;
  Ctx& c = *ctx;
  // host validation first: finite, symmetric in the used (2l+1) block
  if (!D && !c.hub_atoms.empty()) return fail(c, HCU_INVALID_ARG, "null D");
  const int nh = (int)c.hub_atoms.size();
  for (size_t i = 0; i < c.D_in.size(); ++i)
    if (!std::isfinite(D[i])) return fail(c, HCU_NAN, "non-finite entry in D");
  for (int sp = 0; sp < c.p.nspin; ++sp)
    for (int h = 0; h < nh; ++h) {
      const int nm = 2 * c.hub_l[h] + 1;
      const double* d = D + ((size_t)sp * nh + h) * 25;
      for (int i = 0; i < nm; ++i)
        for (int j = i + 1; j < nm; ++j)
          if (std::fabs(d[i * 5 + j] - d[j * 5 + i]) > 1e-12 * (1.0 + std::fabs(d[i * 5 + j])))
            return fail(c, HCU_INVALID_ARG, "D must be symmetric");
    }
  hcu_status s = check_ctx(ctx);
  if (s != HCU_OK) return s;
  for (size_t i = 0; i < c.D_in.size(); ++i) c.D_in[i] = D[i];
  s = upload_coupling(c);
  if (s != HCU_OK) return s;
  HCU_HIP(hipStreamSynchronize(c.stream));
  return HCU_OK;
}

hcu_status hcu_set_start(hcu_ctx* ctx, int spin, int ik, const void* X0, const void* v0) {
  hcu_status s = check_ctx(ctx);
  if (s != HCU_OK) return s;
  Ctx& c = *ctx;
  if (spin < 0 || spin >= c.p.nspin || ik < 0 || ik >= c.p.nk) return fail(c, HCU_INVALID_ARG, "spin/k out of range");
  if (!X0 || !v0) return fail(c, HCU_INVALID_ARG, "null start block");
  const int sk = sk_index(c, spin, ik);
  HCU_HIP(hipMemcpyAsync(c.d_X[sk], X0, esize(c) * (size_t)c.nd * c.p.ns, hipMemcpyDeviceToDevice, c.stream));
  c.px_valid.clear();   // new orbitals: their projections are not at hand
  HCU_HIP(hipMemcpyAsync(c.d_v0[sk], v0, esize(c) * (size_t)c.nd, hipMemcpyDeviceToDevice, c.stream));
  HCU_HIP(hipStreamSynchronize(c.stream));
  return HCU_OK;
}

hcu_status hcu_apply_h(hcu_ctx* ctx, int spin, int ik, const void* X, void* Y, int ncol, int64_t ld) {
  hcu_status s = check_ctx(ctx);
  if (s != HCU_OK) return s;
  Ctx& c = *ctx;
  if (spin < 0 || spin >= c.p.nspin || ik < 0 || ik >= c.p.nk) return fail(c, HCU_INVALID_ARG, "spin/k out of range");
  if (ncol < 1 || ncol > c.p.ns) return fail(c, HCU_INVALID_ARG, "ncol must be in 1..ns");
  if (ld < c.nd) return fail(c, HCU_INVALID_ARG, "ld < nd");
  if (!X || !Y || X == Y) return fail(c, HCU_INVALID_ARG, "bad X/Y pointers");
  return DISPATCH(c, apply_h_v, c, spin, ik, X, Y, ncol, ld);
}

hcu_status hcu_cheb_filter(hcu_ctx* ctx, int spin, int ik, const void* X, void* Y, int ncol, int64_t ld, int m,
                           double a, double b, double aL) {
  hcu_status s = check_ctx(ctx);
  if (s != HCU_OK) return s;
  Ctx& c = *ctx;
  if (spin < 0 || spin >= c.p.nspin || ik < 0 || ik >= c.p.nk) return fail(c, HCU_INVALID_ARG, "spin/k out of range");
  if (ncol < 1 || ncol > c.p.ns) return fail(c, HCU_INVALID_ARG, "ncol must be in 1..ns");
  if (ld < c.nd) return fail(c, HCU_INVALID_ARG, "ld < nd");
  if (!X || !Y || X == Y) return fail(c, HCU_INVALID_ARG, "bad X/Y pointers");
  if (m < 1 || !(aL < a) || !(a < b)) return fail(c, HCU_INVALID_ARG, "need m >= 1 and aL < a < b");
  return DISPATCH(c, filter_v, c, spin, ik, X, Y, ncol, ld, m, a, b, aL);
}

hcu_status hcu_gram(hcu_ctx* ctx, const void* Y, const void* HY, int ncol, int64_t ld, double* S, double* Hs) {
  hcu_status s = check_ctx(ctx);
  if (s != HCU_OK) return s;
  Ctx& c = *ctx;
  if (ncol < 1 || ncol > c.p.ns) return fail(c, HCU_INVALID_ARG, "ncol must be in 1..ns");
  if (ld < c.nd) return fail(c, HCU_INVALID_ARG, "ld < nd");
  if (!Y || !HY || !S || !Hs) return fail(c, HCU_INVALID_ARG, "null pointer");
  return DISPATCH(c, gram_v, c, Y, HY, ncol, ld, S, Hs);
}

hcu_status hcu_rotate(hcu_ctx* ctx, const void* Y, const double* C, void* X, int ncol, int64_t ld) {
  hcu_status s = check_ctx(ctx);
  if (s != HCU_OK) return s;
  Ctx& c = *ctx;
  if (ncol < 1 || ncol > c.p.ns) return fail(c, HCU_INVALID_ARG, "ncol must be in 1..ns");
  if (ld < c.nd) return fail(c, HCU_INVALID_ARG, "ld < nd");
  if (!Y || !C || !X || X == Y) return fail(c, HCU_INVALID_ARG, "bad pointers");
  return DISPATCH(c, rotate_v, c, Y, C, X, ncol, ld);
}

hcu_status hcu_lanczos_bounds(hcu_ctx* ctx, int spin, int ik, int steps, double* theta_min, double* upper) {
  hcu_status s = check_ctx(ctx);
  if (s != HCU_OK) return s;
  Ctx& c = *ctx;
  if (spin < 0 || spin >= c.p.nspin || ik < 0 || ik >= c.p.nk) return fail(c, HCU_INVALID_ARG, "spin/k out of range");
  if (steps < 1 || steps > 200) return fail(c, HCU_INVALID_ARG, "steps must be in 1..200");
  return DISPATCH(c, lanczos_t, c, spin, ik, steps, theta_min, upper);
}

hcu_status hcu_chfsi_pass(hcu_ctx* ctx, int spin, int ik) {
  hcu_status s = check_ctx(ctx);
  if (s != HCU_OK) return s;
  Ctx& c = *ctx;
  if (spin < 0 || spin >= c.p.nspin || ik < 0 || ik >= c.p.nk) return fail(c, HCU_INVALID_ARG, "spin/k out of range");
  const int sk = sk_index(c, spin, ik);
  if (!(c.bounds[3 * sk + 1] > c.bounds[3 * sk])) return fail(c, HCU_INVALID_ARG, "bounds not set (run hcu_lanczos_bounds)");
  return DISPATCH(c, pass_t, c, spin, ik, (double*)nullptr);
}

static hcu_status forces_stress_entry(hcu_ctx* ctx, const double* occ, double* forces, double* stress) {
  hcu_status s = check_ctx(ctx);
  if (s != HCU_OK) return s;
  Ctx& c = *ctx;
  if (!forces && !stress) return fail(c, HCU_INVALID_ARG, "null output");
  if (!occ && !c.have_results)
    return fail(c, HCU_INVALID_ARG, "no occupations yet: run hcu_scf or hcu_update_occupations, or pass occ");
  s = hubbard_forces_stress(c, occ, forces, stress);
  if (s == HCU_NAN) return fail(c, s, "non-finite occupations or results");
  return s;
}

hcu_status hcu_hubbard_forces(hcu_ctx* ctx, const double* occ, double* forces) {
  return forces_stress_entry(ctx, occ, forces, nullptr);
}

hcu_status hcu_hubbard_stress(hcu_ctx* ctx, const double* occ, double* stress) {
  return forces_stress_entry(ctx, occ, nullptr, stress);
}

hcu_status hcu_update_occupations(hcu_ctx* ctx) {
  hcu_status s = check_ctx(ctx);
  if (s != HCU_OK) return s;
  Ctx& c = *ctx;
  return DISPATCH(c, occupations_t, c);
}

hcu_status hcu_scf_begin(hcu_ctx* ctx, const hcu_scf_opts* o) {
  hcu_status s = check_ctx(ctx);
  if (s != HCU_OK) return s;
  Ctx& c = *ctx;
  if (!o) return fail(c, HCU_INVALID_ARG, "null options");
  if (o->max_iter < 1 || o->first_passes < 1 || o->lanczos_steps < 1 || o->pulay_history < 1)
    return fail(c, HCU_INVALID_ARG, "bad SCF options");
  if (c.hxc && (o->pulay_history + 1 > kHxcWindow || !(o->kerker_k0 >= 0) || !std::isfinite(o->kerker_k0) ||
                !(o->tol_rho > 0)))
    return fail(c, HCU_INVALID_ARG, "bad SCF options for the density-dependent Hamiltonian (pulay_history <= 8, "
                                    "kerker_k0 >= 0, tol_rho > 0)");
  s = check_kset(c);
  if (s != HCU_OK) return s;
  c.scf_opts = *o;
  c.scf_iter = 0;
  c.scf_have_old = false;
  c.mix_x.clear();
  c.mix_f.clear();
  c.hxc_slots.clear();
  c.scf_filter_ms = 0;
  c.scf_hx_cols = 0;
  for (int sp = 0; sp < c.p.nspin; ++sp)
    for (int k = 0; k < c.p.nk; ++k) {
      s = DISPATCH(c, lanczos_t, c, sp, k, o->lanczos_steps, (double*)nullptr, (double*)nullptr);
      if (s != HCU_OK) return s;
    }
  c.scf_ready = true;
  return HCU_OK;
}

hcu_status hcu_scf_step(hcu_ctx* ctx, hcu_scf_step_info* info) {
  hcu_status s = check_ctx(ctx);
  if (s != HCU_OK) return s;
  Ctx& c = *ctx;
  if (!c.scf_ready) return fail(c, HCU_INVALID_ARG, "call hcu_scf_begin first");
  const int passes = c.scf_iter == 0 ? c.scf_opts.first_passes : 1;
  const int nsk = c.p.nspin * c.p.nk;
  if (nsk == 1) {
    for (int ps = 0; ps < passes; ++ps) {
      s = DISPATCH(c, pass_t, c, 0, 0, &c.scf_filter_ms);
      if (s != HCU_OK) return s;
    }
  } else {
    // every (spin, k) block of the context in one persistent stencil launch per Chebyshev step
    std::vector<BProb> pr;
    for (int sp = 0; sp < c.p.nspin; ++sp)
      for (int k = 0; k < c.p.nk; ++k) pr.push_back(BProb{&c, sp, k, sk_index(c, sp, k), 0, 0, 0, 0});
    for (int ps = 0; ps < passes; ++ps) {
      s = DISPATCH(c, batch_pass_t, pr, c, &c.scf_filter_ms);
      if (s != HCU_OK) return s;
    }
  }
  c.scf_hx_cols += (double)passes * nsk * c.p.ns * (c.p.degree + 1);
  return scf_post(c, info);
}

hcu_status hcu_scf(hcu_ctx* ctx, const hcu_scf_opts* o, hcu_scf_report* rep) {
  hcu_status s = check_ctx(ctx);
  if (s != HCU_OK) return s;
  Ctx& c = *ctx;
  if (!o || !rep) return fail(c, HCU_INVALID_ARG, "null options/report");
  std::memset(rep, 0, sizeof(*rep));
  const auto t0 = std::chrono::steady_clock::now();
  s = hcu_scf_begin(ctx, o);
  if (s != HCU_OK) return s;
  hcu_status final_status = HCU_NOT_CONVERGED;
  int it = 0;
  hcu_scf_step_info si{};
  for (it = 0; it < o->max_iter; ++it) {
    s = hcu_scf_step(ctx, &si);
    if (s != HCU_OK) return s;
    rep->residual = si.residual;
    rep->residual_rho = si.residual_rho;
    if (o->fixed_iterations > 0) {
      if (it + 1 >= o->fixed_iterations) { final_status = HCU_OK; ++it; break; }
    } else if (si.converged) {
      final_status = HCU_OK;
      rep->converged = 1;
      ++it;
      break;
    }
  }
  rep->iterations = it;
  rep->F = c.en.F;
  rep->E_U = c.en.E_U;
  rep->e_band = c.en.e_band;
  rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  rep->filter_seconds = c.scf_filter_ms * 1e-3;
  rep->hx_columns = c.scf_hx_cols;
  if (final_status != HCU_OK) c.err = "SCF did not converge within max_iter";
  return final_status;
}

hcu_status hcu_autotune(hcu_ctx* ctx, hcu_tuning* best) {
  hcu_status s = check_ctx(ctx);
  if (s != HCU_OK) return s;
  Ctx& c = *ctx;
  return DISPATCH(c, autotune_t, c, best);
}

hcu_status hcu_set_tuning(hcu_ctx* ctx, const hcu_tuning* t) {
  if (!ctx || !t) return HCU_INVALID_ARG;
  Ctx& c = *ctx;
  if (t->tile_x == 0) { c.tile_x = 0; return HCU_OK; }   // back to the built-in choice
  if (!stencil_shape_ok(c, t->tile_x, t->tile_yt, t->ry, t->tile_z, t->halo_ring))
    return fail(c, HCU_INVALID_ARG, "stencil tile shape not admissible for this grid");
  c.tile_x = t->tile_x; c.tile_yt = t->tile_yt; c.ry = t->ry; c.tile_z = t->tile_z; c.halo_ring = t->halo_ring;
  return HCU_OK;
}

hcu_status hcu_get_eigenvalues(const hcu_ctx* ctx, double* eig) {
  if (!ctx || !eig) return HCU_INVALID_ARG;
  if (!ctx->have_results) return HCU_INVALID_ARG;
  std::memcpy(eig, ctx->lam.data(), sizeof(double) * ctx->lam.size());
  return HCU_OK;
}

hcu_status hcu_get_occupations(const hcu_ctx* ctx, double* occ) {
  if (!ctx || !occ) return HCU_INVALID_ARG;
  if (!ctx->have_results) return HCU_INVALID_ARG;
  std::memcpy(occ, ctx->occ.data(), sizeof(double) * ctx->occ.size());
  return HCU_OK;
}

hcu_status hcu_get_hubbard_occupation(const hcu_ctx* ctx, double* D) {
  if (!ctx || (!D && !ctx->D_out.empty())) return HCU_INVALID_ARG;
  if (!ctx->have_results) return HCU_INVALID_ARG;
  std::memcpy(D, ctx->D_out.data(), sizeof(double) * ctx->D_out.size());
  return HCU_OK;
}

hcu_status hcu_get_energies(const hcu_ctx* ctx, hcu_energies* e) {
  if (!ctx || !e) return HCU_INVALID_ARG;
  if (!ctx->have_results) return HCU_INVALID_ARG;
  *e = ctx->en;
  return HCU_OK;
}

hcu_status hcu_get_orbitals(hcu_ctx* ctx, int spin, int ik, void* dst, int on_device) {
  hcu_status s = check_ctx(ctx);
  if (s != HCU_OK) return s;
  Ctx& c = *ctx;
  if (spin < 0 || spin >= c.p.nspin || ik < 0 || ik >= c.p.nk || !dst) return fail(c, HCU_INVALID_ARG, "bad arguments");
  return DISPATCH(c, get_orbitals_v, c, sk_index(c, spin, ik), dst, on_device);
}

hcu_status hcu_get_density(hcu_ctx* ctx, double* rho) {
  hcu_status s = check_ctx(ctx);
  if (s != HCU_OK) return s;
  Ctx& c = *ctx;
  if (!rho) return fail(c, HCU_INVALID_ARG, "null rho");
  if (!c.have_results) return fail(c, HCU_INVALID_ARG, "no occupations yet");
  return DISPATCH(c, density_t, c, rho);
}

hcu_status hcu_get_potential(hcu_ctx* ctx, double* V, double* rho_in) {
  hcu_status s = check_ctx(ctx);
  if (s != HCU_OK) return s;
  Ctx& c = *ctx;
  if (!V) return fail(c, HCU_INVALID_ARG, "null V");
  if (rho_in && !c.hxc) return fail(c, HCU_INVALID_ARG, "no input density without the density-dependent Hamiltonian");
  HCU_HIP(hipMemcpyAsync(V, c.d_V, sizeof(double) * c.nd, hipMemcpyDeviceToHost, c.stream));
  if (rho_in) HCU_HIP(hipMemcpyAsync(rho_in, c.d_rho_in, sizeof(double) * c.nd, hipMemcpyDeviceToHost, c.stream));
  HCU_HIP(hipStreamSynchronize(c.stream));
  return HCU_OK;
}

}  // extern "C"

// ====================================================================== batches
namespace {
hcu_status batch_fail(hcu_batch* b, hcu_status s, const std::string& msg) {
  b->err = msg;
  return s;
}

std::vector<BProb> batch_problems(hcu_batch* b, const std::vector<int>& active) {
  std::vector<BProb> pr;
  for (size_t i = 0; i < b->m.size(); ++i) {
    if (!active[i]) continue;
    Ctx& c = *b->m[i];
    for (int s = 0; s < c.p.nspin; ++s)
      for (int k = 0; k < c.p.nk; ++k) pr.push_back(BProb{&c, s, k, sk_index(c, s, k), 0, 0, 0, 0});
  }
  return pr;
}

hcu_status batch_run_pass(hcu_batch* b, std::vector<BProb>& pr) {
  if (pr.empty()) return HCU_OK;
  Ctx& lead = *pr[0].c;
  hcu_status s = DISPATCH(lead, batch_pass_t, pr, lead, (double*)nullptr);
  if (s != HCU_OK) {
    std::string msg = lead.err;
    for (BProb& q : pr)
      if (!q.c->err.empty()) msg = q.c->err;
    return batch_fail(b, s, msg);
  }
  return HCU_OK;
}
}  // namespace

extern "C" {

hcu_status hcu_batch_create(hcu_ctx* const* ctxs, int n, hcu_batch** out) {
  if (!ctxs || n < 1 || !out) return HCU_INVALID_ARG;
  *out = nullptr;
  hcu_batch* b = new (std::nothrow) hcu_batch();
  if (!b) return HCU_OOM;
  *out = b;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return batch_fail(b, HCU_INVALID_ARG, "null context");
    if (!ctxs[i]->bound) return batch_fail(b, HCU_NOT_BOUND, "every context must be bound");
    b->m.push_back(ctxs[i]);
  }
  const Ctx& c0 = *ctxs[0];
  for (int i = 1; i < n; ++i) {
    const Ctx& c = *ctxs[i];
    if (c.stream != c0.stream) return batch_fail(b, HCU_INVALID_ARG, "contexts must share one stream");
    if (c.mixed != c0.mixed || c.any_complex != c0.any_complex)
      return batch_fail(b, HCU_INVALID_ARG, "contexts must share the block element type");
    if (c.p.degree != c0.p.degree || c.p.n0 != c0.p.n0)
      return batch_fail(b, HCU_INVALID_ARG, "contexts must share the filter degree and FD order");
  }
  return HCU_OK;
}

void hcu_batch_destroy(hcu_batch* b) { delete b; }

const char* hcu_batch_last_error(const hcu_batch* b) { return b ? b->err.c_str() : "null batch"; }

hcu_status hcu_batch_chfsi_pass(hcu_batch* b) {
  if (!b) return HCU_INVALID_ARG;
  for (hcu_ctx* c : b->m)
    for (int sk = 0; sk < c->p.nspin * c->p.nk; ++sk)
      if (!(c->bounds[3 * sk + 1] > c->bounds[3 * sk]))
        return batch_fail(b, HCU_INVALID_ARG, "bounds not set (run hcu_lanczos_bounds on every member)");
  std::vector<int> active(b->m.size(), 1);
  std::vector<BProb> pr = batch_problems(b, active);
  return batch_run_pass(b, pr);
}

hcu_status hcu_batch_scf(hcu_batch* b, const hcu_scf_opts* o, hcu_scf_report* reps) {
  if (!b || !o || !reps) return HCU_INVALID_ARG;
  const size_t nm = b->m.size();
  const auto t0 = std::chrono::steady_clock::now();
  for (size_t i = 0; i < nm; ++i) {
    std::memset(&reps[i], 0, sizeof(hcu_scf_report));
    hcu_status s = hcu_scf_begin(b->m[i], o);
    if (s != HCU_OK) return batch_fail(b, s, b->m[i]->err);
  }
  std::vector<int> active(nm, 1);
  hcu_status final_status = HCU_OK;
  for (int it = 0; it < o->max_iter; ++it) {
    std::vector<BProb> pr = batch_problems(b, active);
    if (pr.empty()) break;
    const int passes = it == 0 ? o->first_passes : 1;
    for (int ps = 0; ps < passes; ++ps) {
      hcu_status s = batch_run_pass(b, pr);
      if (s != HCU_OK) return s;
    }
    for (size_t i = 0; i < nm; ++i) {
      if (!active[i]) continue;
      Ctx& c = *b->m[i];
      c.scf_hx_cols += (double)passes * c.p.nspin * c.p.nk * c.p.ns * (c.p.degree + 1);
      hcu_scf_step_info si{};
      hcu_status s = scf_post(c, &si);
      if (s != HCU_OK) return batch_fail(b, s, c.err);
      reps[i].iterations = it + 1;
      reps[i].residual = si.residual;
      reps[i].residual_rho = si.residual_rho;
      reps[i].F = c.en.F;
      reps[i].E_U = c.en.E_U;
      reps[i].e_band = c.en.e_band;
      reps[i].hx_columns = c.scf_hx_cols;
      const bool done = o->fixed_iterations > 0 ? (it + 1 >= o->fixed_iterations) : (si.converged != 0);
      if (done) {
        active[i] = 0;
        reps[i].converged = o->fixed_iterations > 0 ? 0 : 1;
        reps[i].seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      }
    }
  }
  for (size_t i = 0; i < nm; ++i)
    if (active[i]) {
      reps[i].seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (o->fixed_iterations <= 0) final_status = HCU_NOT_CONVERGED;
    }
  if (final_status != HCU_OK) b->err = "some members did not converge within max_iter";
  return final_status;
}

}  // extern "C"
