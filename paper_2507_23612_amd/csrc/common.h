// Internal declarations of the hubbard_chfsi library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hubbard_chfsi.h"

namespace hcu {

constexpr int kMaxR = 6;        // largest half stencil order handled (FD order 12)
constexpr int kMaxNm = 9;       // functions per projector block (l <= 1 KB: 1+3+... ; Hubbard 2l+1 <= 5)

// ---------------------------------------------------------------- complex
// Interleaved complex with the arithmetic the kernels need.
template <typename R>
struct cplx {
  R re, im;
  __host__ __device__ cplx() : re(0), im(0) {}
  __host__ __device__ cplx(R r) : re(r), im(0) {}
  __host__ __device__ cplx(R r, R i) : re(r), im(i) {}
};
template <typename R> __host__ __device__ inline cplx<R> operator+(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> __host__ __device__ inline cplx<R> operator-(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> __host__ __device__ inline cplx<R> operator*(cplx<R> a, cplx<R> b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
template <typename R> __host__ __device__ inline cplx<R> operator*(R s, cplx<R> a) { return {s * a.re, s * a.im}; }
template <typename R> __host__ __device__ inline cplx<R>& operator+=(cplx<R>& a, cplx<R> b) { a.re += b.re; a.im += b.im; return a; }

template <typename T> struct real_of { using type = T; };
template <typename R> struct real_of<cplx<R>> { using type = R; };

template <typename T> __host__ __device__ inline T conj_(T a) { return a; }
template <typename R> __host__ __device__ inline cplx<R> conj_(cplx<R> a) { return {a.re, -a.im}; }
template <typename T> __host__ __device__ inline typename real_of<T>::type abs2_(T a) { return a * a; }
template <typename R> __host__ __device__ inline R abs2_(cplx<R> a) { return a.re * a.re + a.im * a.im; }
// a * conj(b) accumulate helpers
template <typename T> __host__ __device__ inline T mul_conj(T a, T b) { return a * b; }
template <typename R> __host__ __device__ inline cplx<R> mul_conj(cplx<R> a, cplx<R> b) { return a * conj_(b); }
template <typename T> __host__ __device__ inline T make_scalar(double re, double im) { (void)im; return T(re); }
template <> __host__ __device__ inline cplx<double> make_scalar<cplx<double>>(double re, double im) { return {re, im}; }
template <> __host__ __device__ inline cplx<float> make_scalar<cplx<float>>(double re, double im) { return {float(re), float(im)}; }

// ---------------------------------------------------------------- wave-private LDS hand-off
// Lanes of one wave exchange values through LDS (one lane writes what another
// reads).  The wavefront-scope release/acquire pair orders the LDS write
// before the read (and a read before the next overwrite), and the wave
// barrier keeps the compiler from moving LDS accesses across this point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- XCD-aware order
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  xcd_linear() maps the hardware order to a logical order in which
// each XCD receives a contiguous range of logical indices, so neighbouring
// logical workgroups (that share halo rows or table tiles) share an L2.
constexpr int kNumXcd = 8;
constexpr int kHxcWindow = 9;   // density mixing window: Pulay history of at most 8
__device__ inline unsigned xcd_linear() {
  const unsigned nwg = gridDim.x * gridDim.y * gridDim.z;
  const unsigned w = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const unsigned q = nwg / kNumXcd, r = nwg % kNumXcd;
  const unsigned x = w % kNumXcd, i = w / kNumXcd;
  return x * q + (x < r ? x : r) + i;
}

// Point order of the 64-point bricks of the projector tables.  Linear: brick
// b holds the points 64 b .. 64 b + 63 (the last one cut at the grid end).
// Blocks: brick b is a block of 2^lx x 2^ly x 2^lz grid points (lx >= 2,
// lx + ly + lz = 6) in x-fastest block order, local index
// i = dx + 2^lx (dy + 2^ly dz); a compact block meets the atoms' spherical
// supports more densely than a 64-point run of one grid row.  Local indices
// 4k .. 4k+3 are consecutive in memory in both orders.  Projection brick b
// is made of the bricks 4b .. 4b+3 in either order.
struct BrickGeo {
  int cube = 0;                 // 1: blocks
  int lx = 6, ly = 0, lz = 0;   // log2 of the block edges
  int n1 = 0, nbx = 1, nby = 1;
  int64_t n12 = 0;
  int64_t nbrick = 0;           // bricks of the grid
  __host__ __device__ int64_t base(int64_t b) const {
    if (!cube) return b * 64;
    const int64_t bx = b % nbx, t = b / nbx, by = t % nby, bz = t / nby;
    return (bx << lx) + (int64_t)n1 * (by << ly) + n12 * (bz << lz);
  }
  __host__ __device__ int64_t off(int i) const {
    if (!cube) return i;
    return (i & ((1 << lx) - 1)) + (int64_t)n1 * ((i >> lx) & ((1 << ly) - 1)) + n12 * (i >> (lx + ly));
  }
};

// ---------------------------------------------------------------- context
struct BlockDesc {            // one projector block: the KB channels or the Hubbard manifold of one atom
  int atom;
  int type;                   // 0 = KB, 1 = Hubbard
  int nm;                     // number of functions
  int nsupp;                  // support size
  int64_t supp_off;           // into supp[]
  int64_t val_off;            // into csc values: val[val_off + m*nsupp + q]
  int j0;                     // first global projector index
  int hub;                    // index among Hubbard atoms (type 1), else -1
  int coup_off;               // into coupling matrices (nm*nm doubles)
  // evaluation data
  double center[3];
  int nchan;
  int chan_l[HCU_MAX_KB];
  double chan_rc[HCU_MAX_KB];
  double chan_norm[HCU_MAX_KB];
  double chan_gamma[HCU_MAX_KB];
  double width;               // KB Gaussian width
  int power;                  // Hubbard radial power
  double alpha;               // Hubbard exponent
};

struct StencilCoef {
  int n[3];
  int R;
  double kin[3][kMaxR + 1];   // -1/2 * Laplacian weights per axis, [0] = centre
  double center;              // sum_a kin[a][0]
  double phase_re[3], phase_im[3];   // Bloch factor e^{i k_a L_a}
};

struct Ctx {
  // problem
  hcu_problem p;
  std::vector<double> kpts, kw, pos;
  std::vector<int> atom_species;
  std::vector<hcu_species> species;
  int nd = 0;
  double dv = 0;
  double h[3];
  bool mixed = false;
  bool any_complex = false;
  bool kset_closed = true;           // k-point set closed under k -> -k (equal weights): D is real
  std::vector<int> hub_atoms;        // atom index of each Hubbard atom
  std::vector<int> hub_l;
  std::vector<double> hub_U;
  // projector structure (host)
  std::vector<BlockDesc> blocks;
  std::vector<int> supp;             // concatenated supports
  int nproj = 0;
  int64_t nval = 0;                  // csc values per k
  std::vector<int> csr_ptr, csr_col;
  std::vector<int64_t> csr_src;      // csc position of each csr entry
  int coup_size = 0;
  BrickGeo geo;                      // point order of the bricks
  // Bricks of 64 grid points (geo).  Brick b has bnj[b] functions,
  // listed in bj[boff[b] .. boff[b+1]) (padded to a multiple of 4 with -1),
  // and a dense value tile [slot][64 points].
  std::vector<int64_t> boff;         // nbrick + 1, in slots
  std::vector<int> bnj;
  std::vector<int> bj;
  std::vector<int64_t> bsrc;         // csc position per (slot, point) or -1
  int64_t* d_boff = nullptr;
  int* d_bnj = nullptr;
  int* d_bj = nullptr;
  int64_t* d_bsrc = nullptr;
  std::vector<void*> d_bval;         // per k: [slot][point]
  // Projection bricks (real blocks): runs of kPBrick consecutive points with
  // the union of their functions, laid out like the bricks.  Each slot's
  // partial sum goes to row pdest[slot] of a function-major partial array;
  // function j owns rows jrow[j] .. jrow[j+1] (its bricks in ascending order).
  std::vector<int64_t> pboff;
  std::vector<int> pbnj;
  std::vector<int64_t> pbsrc, pdest, jrow;
  int pgroup = 2;   // points per lane and load group in the table order (2 or 4)
  int max_ptiles = 0;   // most 16-function slot tiles of any projection brick
  int64_t* d_pboff = nullptr;
  int* d_pbnj = nullptr;
  int64_t* d_pbsrc = nullptr;
  int64_t* d_pdest = nullptr;
  int64_t* d_jrow = nullptr;
  std::vector<void*> d_pbval;        // per k: [slot][kPBrick points]
  int nm_count[kMaxNm + 1] = {0};    // projector blocks per function count
  int nm_offset[kMaxNm + 1] = {0};   // offset of each count's list in d_nm_lists
  int* d_nm_lists = nullptr;
  int* d_hub_blocks = nullptr;       // block index of each Hubbard atom
  // device layout (byte offsets into the workspace)
  size_t ws_bytes = 0;
  size_t ws_bound = 0;               // bytes of the bound workspace
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  bool bound = false;
  rocblas_handle blas = nullptr;
  size_t elem = 8;                   // bytes of one block element (real)
  // device pointers
  double* d_V = nullptr;             // V_loc (double)
  float* d_Vf = nullptr;             // V_loc (float, mixed)
  int* d_supp = nullptr;
  BlockDesc* d_blocks = nullptr;
  std::vector<void*> d_cscv;         // per k: csc values (block element type)
  std::vector<double*> d_coup;       // per spin: coupling matrices
  std::vector<void*> d_X;            // per (spin, k): orbitals nd x ns
  std::vector<void*> d_v0;           // per (spin, k): Lanczos start vector
  std::vector<void*> d_W;            // per (spin,k): 3 work blocks nd x ns (index 3 sk + i)
  std::vector<void*> d_P;            // per (spin,k): projections [ns][nproj] (block type)
  std::vector<void*> d_Q;            // per (spin,k): coupled projections, transposed [nproj][ns]
  std::vector<void*> d_PY;           // per (spin,k): projections of the filtered block (for D)
  void* d_jobs = nullptr;            // batched-stencil job table (used when this context leads a batch)
  unsigned long long* d_counters = nullptr;
  void* d_ppart = nullptr;           // projection partial sums [chunk][nproj][ns]
  std::vector<void*> d_ppart_sk;     // per (spin, k) block (several blocks in one fused launch); [0] = d_ppart
  // Hubbard forces and stress
  double* d_lowC = nullptr;          // Loewdin coefficients [nk][nhub][re 25, im 25]
  void* d_momcsc = nullptr;          // moment values on the supports (nval elements)
  void* d_mom[3] = {nullptr, nullptr, nullptr};   // moment tables, projection-brick layout
  void* d_fproj = nullptr;           // 13 projection arrays [ns][nproj]: P, G^a, Q^ab
  double* d_fsum = nullptr;          // per Hubbard atom 325 complex bilinear sums
  double* d_focc = nullptr;          // caller occupations [nspin*nk][ns]
  std::vector<void*> d_PX;           // per (spin,k) projections of X [ns][nproj]
  // per (spin,k): d_PX holds P(X) of the current X and projector tables (set
  // by the Rayleigh-Ritz rotation; cleared when X or the tables are replaced)
  std::vector<unsigned char> px_valid;
  double* d_part = nullptr;          // split-K partials of the Gram matrices
  int2* d_tiles = nullptr;           // upper-triangular output tiles of the Gram kernels
  size_t part_elems = 0;
  double* d_S = nullptr;             // ns x ns (complex: 2x)
  double* d_Hs = nullptr;
  double* d_C = nullptr;             // eigenvectors (ns x ns)
  void* d_Cb = nullptr;              // C in block precision
  double* d_lam = nullptr;           // per (spin,k) eigenvalues [nspin*nk*ns]
  double* d_occ = nullptr;           // per (spin,k) occupations
  double* d_E = nullptr;             // rocsolver work (ns)
  int* d_info = nullptr;
  std::vector<int> h_info_store;     // host copies of the eigensolve status per (spin,k)
  int* h_info = nullptr;             // pinned copy once bound (asynchronous copies from side streams)
  int* h_info_pinned = nullptr;
  // Rayleigh-Ritz steps running beside each other (several blocks): scratch
  // slots 1.. of this context (slot 0 is d_part, d_S, ... above), carved
  // from the workspace, each with its own library handle; side streams and
  // events of the batches this context leads
  struct RRSlot {
    rocblas_handle blas = nullptr;
    double *part = nullptr, *S = nullptr, *Hs = nullptr, *E = nullptr;
    void* Cb = nullptr;
    int* info = nullptr;
  };
  std::vector<RRSlot> rr_slots;
  std::vector<hipStream_t> rr_streams;
  std::vector<hipEvent_t> rr_events;   // [0] main stream, [1 + lane] side streams
  double* d_D = nullptr;             // D_out [nspin][nhub][25]
  double* d_red = nullptr;           // scalar reductions scratch
  double* d_scal = nullptr;          // scalars [0..63]: mu, e_band, dc, E_U, kT S, F, dot results;
                                     // then kw per (spin,k), U per Hubbard atom, coupling pointers
  double* d_rho = nullptr;           // density [nspin][nd]
  void* d_vec = nullptr;             // Lanczos work vectors (4 x nd)
  // state
  std::vector<double> D_in;          // [nspin][nhub][25]
  std::vector<double> bounds;        // per (spin,k): a, b, aL
  std::vector<double> lam;           // host copy of eigenvalues
  std::vector<double> occ;
  std::vector<double> D_out;
  hcu_energies en{};
  bool have_results = false;
  // density-dependent Hamiltonian (problem flag hxc): d_V holds V_loc + V_H + V_x
  bool hxc = false;
  bool hxc_have_rho = false;         // d_rho_in holds an input density
  double* d_Vloc = nullptr;          // V_loc alone
  double* d_rho_in = nullptr;        // input density of the current iteration
  double* d_hx = nullptr;            // mixing window: input densities [kHxcWindow][nd]
  double* d_hf = nullptr;            // mixing window: residuals [kHxcWindow][nd]
  double* d_hbar = nullptr;          // two grid vectors of the mixing step
  double* d_hspec = nullptr;         // two half spectra [2][n3][n2][n1/2+1] complex
  double* d_hsym = nullptr;          // -Delta_h symbol per axis [n1/2+1 | n2 | n3]
  double* d_hpart = nullptr;         // reduction partials
  std::vector<int> hxc_slots;        // window slots in use, oldest first
  double hxc_res = 0;                // density residual of the last energies
  void* hxc_plan[2] = {nullptr, nullptr};   // FFT plans: real to complex, complex to real
  // AIMD history: positions and converged D of the last geometries, most recent first
  std::vector<std::vector<double>> aimd_pos, aimd_D;
  std::string err;
  // tuning
  int tile_x = 0, tile_yt = 0, ry = 4, tile_z = 0, halo_ring = 0;
  // SCF state (hcu_scf_begin / hcu_scf_step)
  hcu_scf_opts scf_opts{};
  int scf_iter = 0;
  bool scf_ready = false;
  double scf_F_old = 0;
  bool scf_have_old = false;
  std::vector<std::vector<double>> mix_x, mix_f;
  double scf_filter_ms = 0;
  double scf_hx_cols = 0;
  // kernel timing (HIP events on the bound stream, resolved at sync points)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  double prof_ms[8] = {0};
  long prof_count[8] = {0};
};

enum ProfKind { PK_STENCIL = 0, PK_PROJECT = 1, PK_GRAM = 2, PK_EIG = 3, PK_ROTATE = 4, PK_SCATTER = 5,
                PK_FUSED = 6, PK_HXC = 7 };

// Scoped timing of the launches queued inside it (no-op unless profiling).
// Per-phase GPU time.  A marker event recorded between two kernels on a
// stream can be timestamped before the earlier kernel has drained, so phases
// made of our own kernels take the begin and end timestamps of the kernels'
// own dispatches instead (launch_k below: the first kernel of the phase
// stamps its start, every kernel re-stamps the stop).  Phases made of
// library calls (the eigensolve) fall back to marker events.
struct KTimer {
  hipEvent_t start = nullptr, stop = nullptr;
  bool started = false;
};
extern thread_local KTimer* g_ktimer;

template <typename K, typename... A>
inline void launch_k(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t st, A... args) {
  KTimer* t = g_ktimer;
  if (!t) {
    kernel<<<grid, block, lds, st>>>(args...);
    return;
  }
  hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, st, t->started ? nullptr : t->start, t->stop, 0u,
                        args...);
  t->started = true;
}

struct ProfScope {
  Ctx& c;
  int kind;
  bool markers;
  KTimer t, *saved = nullptr;
  ProfScope(Ctx& c_, int k, bool library_calls = false) : c(c_), kind(k), markers(library_calls) {
    if (!c.prof) return;
    t.start = take();
    t.stop = take();
    if (markers) {
      (void)hipEventRecord(t.start, c.stream);
    } else {
      saved = g_ktimer;
      g_ktimer = &t;
    }
  }
  ~ProfScope() {
    if (!c.prof) return;
    if (markers) {
      (void)hipEventRecord(t.stop, c.stream);
    } else {
      g_ktimer = saved;
      if (!t.started) {   // nothing launched in this phase
        c.ev_pool.push_back(t.start);
        c.ev_pool.push_back(t.stop);
        return;
      }
    }
    c.ev_pending.push_back({kind, {t.start, t.stop}});
  }
  hipEvent_t take() {
    hipEvent_t e;
    if (!c.ev_pool.empty()) { e = c.ev_pool.back(); c.ev_pool.pop_back(); }
    else (void)hipEventCreate(&e);
    return e;
  }
};
void prof_resolve(Ctx& c);
// the density of the current orbitals and occupations into d_rho (api.hip)
hcu_status compute_density(Ctx& c);   // after a stream sync: accumulate and recycle events

inline int sk_index(const Ctx& c, int spin, int ik) { return spin * c.p.nk + ik; }
inline bool k_complex(const Ctx& c, int ik) {
  return c.kpts[3 * ik] != 0.0 || c.kpts[3 * ik + 1] != 0.0 || c.kpts[3 * ik + 2] != 0.0;
}

// ---------------------------------------------------------------- launchers
// setup.hip
hcu_status build_structure(Ctx& c);          // host: supports, blocks, csr
hcu_status device_tables(Ctx& c);            // device: V_loc, csc/csr values, Loewdin
void fill_stencil_coef(const Ctx& c, int ik, StencilCoef& sc);

// eig.hip: Householder tridiagonalization of the Rayleigh-Ritz matrix in one workgroup
bool sytrd_small_ok(int n);
void launch_sytrd_small(double* A, int n, int lda, double* d, double* e, double* tau, hipStream_t st);
bool hetrd_small_ok(int n);
void launch_hetrd_small(cplx<double>* A, int n, int lda, double* d, double* e, cplx<double>* tau, hipStream_t st);

// hxc.hip: the density-dependent potential and the mixing of the density
size_t hxc_spectrum_elems(const Ctx& c);
size_t hxc_partial_elems();
hcu_status hxc_after_structure(Ctx& c);     // symbol tables, FFT plans, potential
hcu_status hxc_reset_density(Ctx& c);       // uniform rho_in, empty window, potential
hcu_status hxc_refresh_potential(Ctx& c);   // V from rho_in
hcu_status hxc_energies(Ctx& c);            // of the output density in d_rho
hcu_status hxc_mix(Ctx& c, int hist, double beta, double k0, std::vector<double>& gamma);
void hxc_destroy(Ctx& c);

// stencil.hip: out = alpha*(H_loc y - c y) - beta*yprev
template <typename T>
void launch_stencil(const Ctx& c, int ik, const T* Yin, int64_t ld, const T* Yprev, int64_t ld_prev, T* Yout,
                    int64_t ld_out, int ncol, double alpha, double cshift, double beta, hipStream_t st);
bool stencil_shape_ok(const Ctx& c, int TX, int TYt, int RY, int tz, int ring);
// one block of a batched stencil step (stencil.hip, persistent launch)
struct StencilJob {
  const Ctx* c;
  int ik;
  const void* Yin;
  int64_t ld;
  const void* Yprev;
  int64_t ld_prev;
  void* Yout;
  int64_t ld_out;
  int ncol;
  double alpha, cshift, beta;
};
// Persistent stencil launches over many blocks, planned ahead: plan appends
// the job records of one step (grouped by tile shape, one launch per group)
// to `host` and the launches to `out`; after the caller has copied `host` to
// the device job table, run issues one planned launch: persistent (fixed
// grid draining per-XCD counters) when d_counters is given, else one
// workgroup per work item.
struct BatchLaunch {
  size_t first;                 // first job record of the launch
  int njob;
  unsigned long long total;     // work items
  int TX, TYt, RY, R;
  int halo_slots;               // most halo values per thread and plane over the jobs
  int ring;                     // halo ring (order-12 stencil only)
  int halo_n;                   // most halo values per plane over the jobs
};
template <typename T>
hcu_status plan_stencil_batch(const std::vector<StencilJob>& jobs, std::vector<unsigned char>& host,
                              std::vector<BatchLaunch>& out);
template <typename T>
hcu_status run_stencil_batch(const BatchLaunch& L, const void* d_jobs, unsigned long long* d_counters,
                             hipStream_t st);
// nonlocal.hip: Y += alpha * sum_j phi_j Qt[j][s]  (64-point bricks on the
// matrix cores)
template <typename T>
void launch_nl_scatter(const Ctx& c, int ik, T* Y, int64_t ld, int ncol, const T* Qt, double alpha, hipStream_t st);
constexpr int kBrick = 64;
constexpr int kRRLanes = 4;   // Rayleigh-Ritz steps of different blocks in flight at once
constexpr int kPBrick = 256;

// 16x16x4 matrix-core step D += A B per wave.  Operands: lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; result column l%16, rows row(l, r).
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
template <typename T> struct Mf;
template <> struct Mf<double> {
  using V = d4;
  __device__ static inline V mfma(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mf<float> {
  using V = f4;
  __device__ static inline V mfma(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// proj.hip: P = Phi^H Y dV and Q = C_b P (transposed)
// per-brick partials on the matrix cores (every point of the block read
// once), then per-function sums over the function's slots.
template <typename T>
void launch_project_brick(const Ctx& c, int ik, const T* Y, int ncol, int64_t ld, const double* coup, T* P, T* Q,
                          hipStream_t st);
size_t project_partial_elems(const Ctx& c);
// Q = C P (the coupling alone, for projections already at hand)
template <typename T>
void launch_couple(const Ctx& c, const T* P, int ncol, const double* coup, T* Q, hipStream_t st);
// projections only (no coupling) with a caller-chosen function table in the
// projection-brick layout
template <typename T>
void launch_project_table(const Ctx& c, const T* table, const T* Y, int ncol, int64_t ld, T* P, hipStream_t st);
// setup.hip: moment functions sum_T phi(x-R-T)(x-R-T)_b e^{ik.T} of the
// Hubbard orbitals (orbitals' Loewdin coefficients applied) in the
// projection-brick layout; csc: scratch of nval elements
template <typename T>
hcu_status build_moment_table(Ctx& c, int ik, int b, T* csc, T* table, hipStream_t st);
// Real blocks: Y += alpha Phi Q and, in the same pass, P and Q of the
// updated Y (the next Chebyshev step's input); usable when scatter_project_ok.
template <typename T>
bool scatter_project_ok(const Ctx& c);
// The fused pass of several blocks in one launch: one record per block,
// workgroups item0 .. of each job (jobs ordered by item0).
struct FusedJob {
  BrickGeo geo;
  void* Y; int64_t ld; int ncol; int nst;
  const int64_t* boff; const int* bnj; const int* bj; const void* bval;
  const void* Qt; int ldq; double alpha; int nbrick;
  const int64_t* pboff; const int* pbnj; const void* pbval; const int64_t* pdest;
  void* part; int ldp; int64_t nd;
  unsigned item0;
};
template <typename T>
FusedJob fused_job_of(const Ctx& c, int ik, T* Y, int64_t ld, int ncol, const T* Qt, double alpha, void* part,
                      unsigned item0);
unsigned fused_job_items(const Ctx& c, int ncol);
template <typename T>
void launch_scatter_project_batch(const FusedJob* d_jobs, int njob, unsigned items, int G, int NT, hipStream_t st);
template <typename T>
void launch_scatter_project(const Ctx& c, int ik, T* Y, int64_t ld, int ncol, const T* Qt, double alpha,
                            const double* coup, T* P, T* Q, hipStream_t st, int part = 3);

// forces.hip: Hubbard forces [natom][3] and/or stress [3][3] of the current
// orbitals with the given occupations (host [nspin][nk][ns], NULL = the
// context's); either output may be NULL
hcu_status hubbard_forces_stress(Ctx& c, const double* occ, double* forces, double* stress);

// gemm.hip
size_t gram_partial_elems(int n, int64_t nd);
size_t gram_partial_elems_c(int n, int64_t nd);
std::vector<int2> gram_tiles(int n, bool cplx_);
template <typename T>
void launch_gram2(const Ctx& c, const T* Y, const T* HY, int ncol, int64_t ld, double* S, double* Hs,
                  hipStream_t st);
// the same contraction with caller-given scratch of gram_scratch_bytes()
// (partials, then the tile list); no context
size_t gram_scratch_bytes(int ncol, int64_t nd, bool cplx_);
void launch_gram_scratch(const void* Y, const void* HY, int ncol, int64_t ld, int64_t nd, double dv, bool fp32,
                         bool cplx_, void* scratch, double* S, double* Hs, hipStream_t st);
template <typename T>
void launch_rotate(const Ctx& c, const T* Y, int64_t ld, const T* Cb, T* X, int ncol, hipStream_t st);
template <typename T>
void launch_rotate_proj(const Ctx& c, const T* PY, const T* Cb, T* PX, int ncol, hipStream_t st);

// scf_kernels.hip
template <typename T>
void launch_dot(const Ctx& c, const T* x, const T* y, int64_t n, double* out2, hipStream_t st);
template <typename T>
void launch_axpby(const Ctx& c, T* y, const T* x, double a_re, double a_im, double b, int64_t n, hipStream_t st);
template <typename T>
void launch_scale_copy(T* dst, const T* src, double s, int64_t n, hipStream_t st);
template <typename T>
void launch_convert_c(const double* C, T* Cb, int n, int cplx, hipStream_t st);
void launch_fermi(const Ctx& c, hipStream_t st);
template <typename T>
void launch_occupation_matrix(const Ctx& c, int spin, int ik, const T* PX, hipStream_t st);
void launch_energies(const Ctx& c, const double* d_coup_all, hipStream_t st);
// guards of the projected eigenproblem (info[2]: non-finite S or Hs;
// info[0] != 0: failed Cholesky); both replace the matrices by the identity
void launch_rr_guard_in(double* S, double* Hs, int n, int cp, int* info, hipStream_t st);
void launch_rr_guard_chol(double* U, double* Hs, int n, int cp, const int* info, hipStream_t st);
template <typename T>
void launch_density(const Ctx& c, const T* X, int64_t ld, const double* occ, double w, double* rho,
                    hipStream_t st);

}  // namespace hcu

// the opaque handle of the C ABI
struct hcu_ctx : public hcu::Ctx {};


#define HCU_HIP_CTX(ctx, call)                                               \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) {                                                  \
      (ctx).err = std::string("HIP error: ") + hipGetErrorString(e_);         \
      return HCU_DEVICE;                                                     \
    }                                                                        \
  } while (0)

#define HCU_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) {                                                  \
      c.err = std::string("HIP error: ") + hipGetErrorString(e_) + " at " +  \
              __FILE__ + ":" + std::to_string(__LINE__);                     \
      return HCU_DEVICE;                                                     \
    }                                                                        \
  } while (0)
