// Local part of H and the Chebyshev three-term step in one pass over the grid:
//
//   out = alpha * ( -1/2 Delta_h y + V y - c y ) - beta * yprev
//
// -1/2 Delta_h is the centred 2*n0-order stencil along each axis with
// periodic wrap and the Bloch factor e^{+-i k_a L_a} on wrapped values
// (Sec. II.B: off-grid indices are mapped back periodically with the Bloch
// factor).  The projector term alpha * sum_j phi_j Q_j is added afterwards by
// the state-blocked scatter kernel (nonlocal.hip).
//
// Layout: y is one column of an nd x ncol column-major block, x fastest.  A
// workgroup owns a TX x TY tile of an x-y plane for one state and streams a
// range of z planes; each thread owns RY points stacked in y and keeps the
// 2R+1 z-neighbours of each in registers.  The current plane (with its x/y
// halo, wrapped) is staged in LDS; x and y neighbours come from LDS, z
// neighbours from the register queue.
#include "common.h"

#include <algorithm>
#include <type_traits>

namespace hcu {


template <typename RT>
struct KArgs {
  RT kx[kMaxR + 1], ky[kMaxR + 1], kz[kMaxR + 1];
  RT center;                    // sum of the three centre weights
  RT alpha, cshift, beta;
  RT ph_re[3], ph_im[3];        // Bloch factor per axis
  int n1, n2, n3;
  int tiles_x, tz;
  int has_prev;
  int64_t ld, ld_prev, ld_out;
};

template <typename RT>
struct SJob {
  const void* Yin;
  const void* Yprev;
  void* Yout;
  const RT* V;
  KArgs<RT> a;
  int ntiles, nzc;
  unsigned long long item_begin;
};

// global-memory pointer (job records hold generic pointers; the explicit
// address space keeps the accesses global rather than flat)
template <typename T> using gptr = __attribute__((address_space(1))) T*;

// element access through generic or global pointers (complex values by
// components: the class type has no address-space-qualified copy)
template <typename T> __device__ inline T ldv(const T* p, int64_t i) { return p[i]; }
template <typename T> __device__ inline T ldv(gptr<const T> p, int64_t i) { return p[i]; }
template <typename R> __device__ inline cplx<R> ldv(gptr<const cplx<R>> p, int64_t i) {
  const gptr<const R> q = (gptr<const R>)p;
  return cplx<R>(q[2 * i], q[2 * i + 1]);
}
template <typename T> __device__ inline void stv(gptr<T> p, int64_t i, T v) { p[i] = v; }
template <typename R> __device__ inline void stv(gptr<cplx<R>> p, int64_t i, cplx<R> v) {
  const gptr<R> q = (gptr<R>)p;
  q[2 * i] = v.re;
  q[2 * i + 1] = v.im;
}

// Bloch factor of a node reached with wrap counts w (each -1, 0, 1) applied
// to its value: identity for real blocks.
template <typename T> struct Ph {
  template <typename RT>
  __device__ static inline T apply(T v, int wx, int wy, int wz, const KArgs<RT>&) {
    (void)wx; (void)wy; (void)wz;
    return v;
  }
};
template <typename R> struct Ph<cplx<R>> {
  template <typename RT>
  __device__ static inline cplx<R> apply(cplx<R> v, int wx, int wy, int wz, const KArgs<RT>& a) {
    // the phase first, then one product (by 1 for an unwrapped node)
    cplx<R> ph(R(1), R(0));
    const int w[3] = {wx, wy, wz};
    for (int d = 0; d < 3; ++d) {
      const cplx<R> f(a.ph_re[d], w[d] > 0 ? a.ph_im[d] : -a.ph_im[d]);
      for (int t = 0; t < (w[d] > 0 ? w[d] : -w[d]); ++t) ph = ph * f;
    }
    return v * ph;
  }
};
// value of the (possibly wrapped) node
template <typename T> struct Ld {
  template <typename RT, typename PT>
  __device__ static inline T get(PT y, int64_t idx, int wx, int wy, int wz, const KArgs<RT>& a) {
    return Ph<T>::apply(ldv(y, idx), wx, wy, wz, a);
  }
};

// periodic image of grid coordinate g: returns g - w n in [0, n), w = floor(g / n)
__device__ inline int wrap(int g, int n, int& w) {
  w = (g >= 0) ? g / n : -((n - 1 - g) / n);
  return g - w * n;
}

// Halo values a thread stages per plane (host checks the bound).  Kernels
// come with 8 slots and, for the single-block and persistent forms, with 4:
// the slot bookkeeping lives in registers, and most tiles need at most 4.
constexpr int kHaloSlots = 8;
constexpr int kHaloSlotsSmall = 4;

// Halo ring (HR): a tile reads its neighbours' rows of plane q at the time
// it reads its own rows of plane q as queue head, R planes before it
// computes plane q, so that the neighbour tiles' reads of the same rows
// (their own queue heads) fall in the same time window and meet in L2.  The
// halo values wait in a thread-private LDS ring of R planes until the plane
// is staged; without the ring they are read R planes later than the
// neighbours read them, when the rows have mostly left L2.
constexpr int kRingR = 6;   // the ring is built for the order-12 stencil

// One work item: tile `tile` of the x-y plane, z chunk `zc`, state `s`.
template <typename T, typename RT, int R, int RY, int NHS, bool HR = false>
__device__ __forceinline__ void stencil_item(const T* __restrict__ Yin, const T* __restrict__ Yprev,
                                             T* __restrict__ Yout, const RT* __restrict__ V, const KArgs<RT>& a,
                                             int tile, int zc, int64_t s, unsigned char* smem_raw) {
  const int TX = blockDim.x, TYt = blockDim.y, TY = TYt * RY;
  const int SW = TX + 2 * R, SH = TY + 2 * R;
  T* const buf0 = reinterpret_cast<T*>(smem_raw);
  T* const buf1 = buf0 + SW * SH;
  T* const ring = buf1 + SW * SH;   // HR: [plane mod R][halo value e]
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = ty * TX + tx, nthr = TX * TYt;
  const int bx = tile % a.tiles_x, by = tile / a.tiles_x;
  const int x0 = bx * TX, y0 = by * TY;
  const int zbeg = zc * a.tz;
  const int zend = min(zbeg + a.tz, a.n3);
  // Real FP32 blocks: tiles of odd checkerboard parity sweep their z range
  // R planes behind the even ones (periodic in z, so only the starting
  // plane moves).  A tile reads its own rows of plane q as queue head while
  // its output plane is q - R, and its neighbours' rows of plane q as halo
  // while its output plane is q; with the shift the lagging tile's head
  // reads coincide in time with the leading tile's halo reads, so half of
  // the halo rows are found in L2 (9 % fewer bytes fetched).  That made
  // the FP32 kernel faster and not the FP64 one, which keeps the plain
  // sweep; so do complex (Bloch) blocks, whose phase factor changes where
  // a sweep crosses the cell.
  constexpr bool kShift = !HR && std::is_same<T, float>::value && std::is_same<RT, float>::value;
  const int zsh = (kShift && ((bx + by) & 1) && a.n3 > R) ? a.n3 - R : 0;
  const gptr<const T> Ys = (gptr<const T>)(Yin + s * a.ld);
  const gptr<const T> Yp = (gptr<const T>)Yprev;
  const gptr<T> Yo = (gptr<T>)Yout;
  const gptr<const RT> Vg = (gptr<const RT>)V;
  const int n1 = a.n1, n2 = a.n2, n3 = a.n3;
  const int64_t plane = (int64_t)n1 * n2;
  // x halo from the LDS row itself when the tile spans the whole x range
  const bool xfull = (TX == n1) && (n1 >= R);

  int wxo, wyo[RY];
  const int gx = wrap(x0 + tx, n1, wxo);
  int gy[RY];
  for (int r = 0; r < RY; ++r) gy[r] = wrap(y0 + ty * RY + r, n2, wyo[r]);

  // halo slots owned by this thread: y halo (2R rows x TX) then, unless
  // xfull, x halo (TY rows x 2R)
  const int nyh = 2 * R * TX, nh = nyh + (xfull ? 0 : TY * 2 * R);
  int h_xy[NHS], h_lds[NHS], h_w[NHS];
  for (int k = 0; k < NHS; ++k) {
    const int e = tid + k * nthr;
    h_lds[k] = -1; h_xy[k] = 0; h_w[k] = 4 * 16 + 4;   // unused: node 0, no wrap
    if (e >= nh) continue;
    int row, col, hx, hy, wx, wy;
    if (e < nyh) {
      const int rh = e / TX;
      col = e % TX + R;
      row = rh < R ? rh : TY + rh;
      hx = wrap(x0 + col - R, n1, wx);
      hy = wrap(y0 + row - R, n2, wy);
    } else {
      const int e2 = e - nyh;
      const int cc = e2 % (2 * R);
      row = e2 / (2 * R) + R;
      col = cc < R ? cc : TX + cc;
      hx = wrap(x0 + col - R, n1, wx);
      hy = wrap(y0 + row - R, n2, wy);
    }
    h_lds[k] = row * SW + col;
    h_xy[k] = hx + n1 * hy;
    h_w[k] = (wx + 4) * 16 + (wy + 4);
  }
  // halo values of a plane (the ring holds nh per plane; slot k of this
  // thread is value e = tid + k * nthr)

  T q[RY][2 * R + 1];
  for (int dz = -R; dz <= R; ++dz) {
    int wz;
    const int gz = wrap(zbeg + zsh + dz, n3, wz);
    for (int r = 0; r < RY; ++r)
      q[r][dz + R] = Ld<T>::get(Ys, gx + (int64_t)n1 * gy[r] + plane * gz, wxo, wyo[r], wz, a);
  }
  // stage plane zbeg
  // Halo values are loaded raw and take their Bloch factor when staged
  // (hwz: the plane's z wrap count): a product right after the loads would
  // make the wave wait for them before computing the current plane.
  auto stage = [&](T* buf, const T* hreg, int hwz) {
    for (int r = 0; r < RY; ++r) {
      const int row = ty * RY + r + R;
      const T v = q[r][R];
      buf[row * SW + tx + R] = v;
      if (xfull) {
        if (tx < R) buf[row * SW + tx + n1 + R] = Ph<T>::apply(v, 1, 0, 0, a);
        if (tx >= n1 - R) buf[row * SW + tx - n1 + R] = Ph<T>::apply(v, -1, 0, 0, a);
      }
    }
    for (int k = 0; k < NHS; ++k)
      if (h_lds[k] >= 0) buf[h_lds[k]] = Ph<T>::apply(hreg[k], h_w[k] / 16 - 4, h_w[k] % 16 - 4, hwz, a);
  };
  T hreg[NHS];
  {
    int wz;
    const int gz = wrap(zbeg + zsh, n3, wz);
    // unused slots load node 0 of the plane too (never staged): a guarded
    // load would end in a wait before the next one issues
    for (int k = 0; k < NHS; ++k) hreg[k] = ldv(Ys, h_xy[k] + plane * gz);
    stage(buf0, hreg, wz);
    if constexpr (HR) {
      // halo of planes zbeg+1 .. zbeg+R (clamped to the range: the ones past
      // its end are never staged) into ring planes (p - zbeg) mod R, in two
      // batches of loads (all R at once would raise the register peak)
      constexpr int kB = (R + 1) / 2;
      for (int j0 = 1; j0 <= R; j0 += kB) {
        T hp[kB][NHS];
        for (int j = 0; j < kB; ++j) {
          const int64_t pz = plane * min(zbeg + min(j0 + j, R), zend - 1);
          for (int k = 0; k < NHS; ++k) hp[j][k] = ldv(Ys, h_xy[k] + pz);
        }
        for (int j = 0; j < kB && j0 + j <= R; ++j)
          for (int k = 0; k < NHS; ++k)
            if (tid + k * nthr < nh) ring[((j0 + j) % R) * nh + tid + k * nthr] = hp[j][k];
      }
    }
  }
  __syncthreads();
  int rs = R == 1 ? 0 : 1;   // HR: ring slot of plane z + 1

  int cur = 0;
  for (int z = zbeg; z < zend; ++z) {
    const bool more = z + 1 < zend;
    // prefetch: next plane's halo and queue head, this plane's V and Yprev
    // (raw values: the queue head takes its Bloch factor when it enters the
    // queue, the halo when staged)
    T qn[RY];
    int wzn = 0;
    if (more) {
      const int gz = wrap(z + 1 + R + zsh, n3, wzn);
      for (int r = 0; r < RY; ++r) qn[r] = ldv(Ys, gx + (int64_t)n1 * gy[r] + plane * gz);
      // HR: the halo of plane z + 1 + R, with the queue head (clamped to
      // the range: the planes past its end are never staged)
      const int zh = HR ? min(z + 1 + R, zend - 1) : z + 1 + zsh - (z + 1 + zsh >= n3 ? n3 : 0);
      for (int k = 0; k < NHS; ++k) hreg[k] = ldv(Ys, h_xy[k] + plane * zh);   // unused slots: node 0
    }
    const int64_t zoff = plane * (z + zsh - (z + zsh >= n3 ? n3 : 0));
    RT vv[RY];
    T yp[RY];
    for (int r = 0; r < RY; ++r) {
      const int64_t pidx = gx + (int64_t)n1 * gy[r] + zoff;
      vv[r] = Vg[pidx];
      yp[r] = T(0);
      if (a.has_prev) yp[r] = ldv(Yp, s * a.ld_prev + pidx);
    }
    const T* B = cur ? buf1 : buf0;
    for (int r = 0; r < RY; ++r) {
      const int row = ty * RY + r + R;
      const T* L = B + row * SW + tx + R;
      T acc = T(0);
      for (int p = 1; p <= R; ++p) {
        acc += a.kx[p] * (L[p] + L[-p]);
        // y neighbours inside the thread's own RY rows come from the queue
        // centres (the same values the plane buffer holds)
        const T up = (r + p < RY) ? q[(r + p) % RY][R] : L[p * SW];
        const T dn = (r - p >= 0) ? q[(r - p + RY) % RY][R] : L[-p * SW];
        acc += a.ky[p] * (up + dn);
        acc += a.kz[p] * (q[r][R + p] + q[r][R - p]);
      }
      const bool active = (x0 + tx < n1) && (y0 + ty * RY + r < n2);
      if (active) {
        const int64_t pidx = gx + (int64_t)n1 * gy[r] + zoff;
        acc += (a.center + vv[r] - a.cshift) * q[r][R];
        T out = a.alpha * acc;
        if (a.has_prev) out += (-a.beta) * yp[r];
        stv(Yo, s * a.ld_out + pidx, out);
      }
    }
    for (int r = 0; r < RY; ++r) {
      for (int t = 0; t < 2 * R; ++t) q[r][t] = q[r][t + 1];
      if (more) q[r][2 * R] = Ph<T>::apply(qn[r], wxo, wyo[r], wzn, a);
    }
    if (more) {
      if constexpr (HR) {
        // plane z + 1 leaves its ring slot, plane z + 1 + R takes it (the
        // same thread's entries: no barrier between the two)
        T hv[NHS];
        for (int k = 0; k < NHS; ++k) {
          hv[k] = hreg[k];
          if (tid + k * nthr < nh) {
            T* const e = ring + rs * nh + tid + k * nthr;
            hv[k] = *e;
            *e = hreg[k];
          }
        }
        stage(cur ? buf0 : buf1, hv, 0);
        rs = rs + 1 == R ? 0 : rs + 1;
      } else {
        stage(cur ? buf0 : buf1, hreg, 0);
      }
    }
    __syncthreads();
    cur ^= 1;
  }
}

template <typename T, typename RT, int R, int RY, int NHS, bool HR = false>
__global__ __launch_bounds__(512) void k_stencil(const T* __restrict__ Yin, const T* __restrict__ Yprev,
                                                 T* __restrict__ Yout, const RT* __restrict__ V,
                                                 const KArgs<RT> a) {
  extern __shared__ unsigned char smem_raw[];
  // logical order: tile fastest, then z chunk, then state; XCD-contiguous
  const unsigned lw = xcd_linear();
  const int tile = lw % gridDim.x;
  const int zc = (lw / gridDim.x) % gridDim.y;
  const int64_t s = lw / (gridDim.x * gridDim.y);
  stencil_item<T, RT, R, RY, NHS, HR>(Yin, Yprev, Yout, V, a, tile, zc, s, smem_raw);
}

// Large-workgroup form (up to 1024 threads, e.g. a 72 x 12 tile with one
// point per thread): fewer halo rows per tile row at the price of a
// 128-register budget, so only the light variants (real blocks, RY = 1 in
// FP64, RY <= 2 in FP32) use it.
template <typename T, typename RT, int R, int RY>
__global__ __launch_bounds__(1024) void k_stencil_big(const T* __restrict__ Yin, const T* __restrict__ Yprev,
                                                      T* __restrict__ Yout, const RT* __restrict__ V,
                                                      const KArgs<RT> a) {
  extern __shared__ unsigned char smem_raw[];
  const unsigned lw = xcd_linear();
  const int tile = lw % gridDim.x;
  const int zc = (lw / gridDim.x) % gridDim.y;
  const int64_t s = lw / (gridDim.x * gridDim.y);
  stencil_item<T, RT, R, RY, kHaloSlots>(Yin, Yprev, Yout, V, a, tile, zc, s, smem_raw);
}

// Persistent form over a list of jobs (blocks of possibly different grids):
// the item space [0, total) is cut into kNumXcd contiguous ranges with one
// counter each; workgroup w starts on range w % kNumXcd (the XCD it runs on)
// and moves to the next range when its own is exhausted.  Every workgroup
// leaves after visiting all ranges, so the grid always drains.
template <typename T, typename RT, int R, int RY, int NHS, bool HR = false>
__global__ __launch_bounds__(512) void k_stencil_batch(const SJob<RT>* __restrict__ jobs, int njobs,
                                                       unsigned long long total,
                                                       unsigned long long* __restrict__ counters) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ unsigned long long s_item;
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const unsigned long long per = (total + kNumXcd - 1) / kNumXcd;
  const int r0 = (int)(blockIdx.x % kNumXcd);
  for (int rr = 0; rr < kNumXcd; ++rr) {
    const int r = (r0 + rr) % kNumXcd;
    const unsigned long long lo = per * r;
    const unsigned long long hi = min(total, lo + per);
    for (;;) {
      if (tid == 0) s_item = lo + atomicAdd(&counters[r], 1ULL);
      __syncthreads();
      // the item is the same for the whole workgroup: make it wave-uniform so
      // the job record is read into scalar registers
      const unsigned long long it = s_item;
      const unsigned long long item =
          ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(it >> 32)) << 32) |
          (unsigned)__builtin_amdgcn_readfirstlane((unsigned)it);
      __syncthreads();
      if (item >= hi) break;
      int j = 0;
      while (j + 1 < njobs && jobs[j + 1].item_begin <= item) ++j;
      j = __builtin_amdgcn_readfirstlane(j);
      const SJob<RT>& jb = jobs[j];
      const unsigned long long loc = item - jb.item_begin;
      const int tile = (int)(loc % jb.ntiles);
      const int zc = (int)((loc / jb.ntiles) % jb.nzc);
      const int64_t s = (int64_t)(loc / ((unsigned long long)jb.ntiles * jb.nzc));
      stencil_item<T, RT, R, RY, NHS, HR>((const T*)jb.Yin, (const T*)jb.Yprev, (T*)jb.Yout, jb.V, jb.a, tile, zc, s,
                                 smem_raw);
    }
  }
}

// Grid form over a list of jobs: one workgroup per work item (job, tile,
// z chunk, state), XCD-contiguous item order, the job found by bisection on
// the items' start indices.  No counters: the hardware dispatcher balances.
template <typename T, typename RT, int R, int RY>
__global__ __launch_bounds__(512) void k_stencil_multi(const SJob<RT>* __restrict__ jobs, int njobs) {
  extern __shared__ unsigned char smem_raw[];
  const unsigned long long item = xcd_linear();
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (jobs[mid].item_begin <= item) lo = mid; else hi = mid - 1;
  }
  const int j = __builtin_amdgcn_readfirstlane(lo);
  const SJob<RT>& jb = jobs[j];
  const unsigned long long loc = item - jb.item_begin;
  const int tile = (int)(loc % jb.ntiles);
  const int zc = (int)((loc / jb.ntiles) % jb.nzc);
  const int64_t s = (int64_t)(loc / ((unsigned long long)jb.ntiles * jb.nzc));
  stencil_item<T, RT, R, RY, kHaloSlots>((const T*)jb.Yin, (const T*)jb.Yprev, (T*)jb.Yout, jb.V, jb.a, tile, zc, s, smem_raw);
}

// Tile shape for a grid: TX threads along x, TYt thread rows, RY points per
// thread along y, tz planes per workgroup.  Tuned values (hcu_autotune) win.
struct StencilShape { int TX, TYt, RY, tz, ring = 0; };

// workgroups above 512 threads run k_stencil_big (128 registers per thread)
static bool big_ok(const Ctx& c, int RY) {
  if (c.any_complex) return false;
  return c.mixed ? RY <= 2 : RY == 1;
}

// halo values per thread and plane for a tile on a grid with n1 points in x
static int halo_slots(int n1, int TX, int TYt, int TY, int R) {
  const int nthr = TX * TYt;
  const int nh = 2 * R * TX + ((TX == n1 && n1 >= R) ? 0 : TY * 2 * R);
  return (nh + nthr - 1) / nthr;
}

// halo values of a plane for a tile on a grid with n1 points in x
static int halo_values(int n1, int TX, int TY, int R) {
  return 2 * R * TX + ((TX == n1 && n1 >= R) ? 0 : TY * 2 * R);
}

// LDS of a workgroup: two staged planes with halo, and the halo ring
// (R planes of halo values) when the tile takes one
static size_t stencil_lds(int n1, int TX, int TYt, int RY, int R, int ring, size_t elem) {
  const int TY = TYt * RY;
  size_t b = 2 * (size_t)(TY + 2 * R) * (TX + 2 * R) * elem;
  if (ring) b += (size_t)R * halo_values(n1, TX, TY, R) * elem;
  return b;
}
constexpr size_t kLdsPerWorkgroup = 160 * 1024;

static bool shape_ok(const Ctx& c, const StencilShape& sh, int R) {
  const int n1 = c.p.n[0], n2 = c.p.n[1];
  if (sh.TX < 1 || sh.TX > n1 || sh.TYt < 1 || sh.TX * sh.TYt > 1024) return false;
  if (sh.TX * sh.TYt > 512 && !big_ok(c, sh.RY)) return false;
  if (sh.RY != 1 && sh.RY != 2 && sh.RY != 4) return false;
  const int TY = sh.TYt * sh.RY;
  if (TY > n2) return false;
  if (halo_slots(n1, sh.TX, sh.TYt, TY, R) > kHaloSlots) return false;
  if (sh.ring) {   // built for the order-12 stencil, 4 halo slots, <= 512 threads
    if (sh.ring != 1 || R != kRingR || sh.TX * sh.TYt > 512) return false;
    if (halo_slots(n1, sh.TX, sh.TYt, TY, R) > kHaloSlotsSmall) return false;
    const size_t elem = c.any_complex ? (c.mixed ? 8 : 16) : (c.mixed ? 4 : 8);
    if (stencil_lds(n1, sh.TX, sh.TYt, sh.RY, R, 1, elem) > kLdsPerWorkgroup) return false;
  }
  return sh.tz >= 1;
}

bool stencil_shape_ok(const Ctx& c, int TX, int TYt, int RY, int tz, int ring) {
  return shape_ok(c, StencilShape{TX, TYt, RY, tz, ring}, c.p.n0);
}

static StencilShape pick_tiles(const Ctx& c, int ncol, int elem) {
  const int n1 = c.p.n[0], n2 = c.p.n[1], n3 = c.p.n[2];
  const int R = c.p.n0;
  StencilShape sh{c.tile_x, c.tile_yt, c.ry, c.tile_z, c.halo_ring};
  if (sh.TX > 0 && shape_ok(c, sh, R)) return sh;
  sh.ring = 0;
  sh.RY = elem > 8 ? 2 : 4;
  sh.TX = n1 <= 128 ? n1 : 64;
  sh.TYt = std::max(1, 256 / sh.TX);
  while (sh.TYt > 1 && sh.TYt * sh.RY > n2) --sh.TYt;
  if (sh.TYt * sh.RY > n2) sh.RY = 2;
  if (sh.TYt * sh.RY > n2) sh.RY = 2, sh.TYt = 1;
  int tiles = ((n1 + sh.TX - 1) / sh.TX) * ((n2 + sh.TYt * sh.RY - 1) / (sh.TYt * sh.RY));
  int zs = 1;
  while ((int64_t)tiles * zs * ncol < 2048 && n3 / (zs * 2) >= 16) zs *= 2;
  sh.tz = (n3 + zs - 1) / zs;
  while (!shape_ok(c, sh, R) && sh.TYt > 1) --sh.TYt;
  return sh;
}

// workgroups above 64 KB of LDS ask for it (gfx950 has 160 KB per CU)
template <typename K>
static void allow_lds(K kernel, size_t lds) {
  if (lds > 65536) (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename T, typename RT, int R>
static void launch_r(int RY, bool small_halo, int ring, const KArgs<RT>& a, dim3 grid, dim3 block, size_t lds,
                     const T* Yin, const T* Yprev, T* Yout, const RT* V, hipStream_t st) {
  if constexpr (R == kRingR) {
    if (ring) {
      auto go = [&](auto kernel) {
        allow_lds(kernel, lds);
        launch_k(kernel, grid, block, lds, st, Yin, Yprev, Yout, V, a);
      };
      if (RY == 4) go(k_stencil<T, RT, R, 4, kHaloSlotsSmall, true>);
      else if (RY == 2) go(k_stencil<T, RT, R, 2, kHaloSlotsSmall, true>);
      else go(k_stencil<T, RT, R, 1, kHaloSlotsSmall, true>);
      return;
    }
  }
  if constexpr (sizeof(T) == sizeof(RT)) {
    if (block.x * block.y > 512) {
      if (RY == 2)
        launch_k(k_stencil_big<T, RT, R, 2>, grid, block, lds, st, Yin, Yprev, Yout, V, a);
      else
        launch_k(k_stencil_big<T, RT, R, 1>, grid, block, lds, st, Yin, Yprev, Yout, V, a);
      return;
    }
  }
  auto go = [&](auto nhs) {
    constexpr int NHS = decltype(nhs)::value;
    if (RY == 4)
      launch_k(k_stencil<T, RT, R, 4, NHS>, grid, block, lds, st, Yin, Yprev, Yout, V, a);
    else if (RY == 2)
      launch_k(k_stencil<T, RT, R, 2, NHS>, grid, block, lds, st, Yin, Yprev, Yout, V, a);
    else
      launch_k(k_stencil<T, RT, R, 1, NHS>, grid, block, lds, st, Yin, Yprev, Yout, V, a);
  };
  if (small_halo) go(std::integral_constant<int, kHaloSlotsSmall>());
  else go(std::integral_constant<int, kHaloSlots>());
}

template <typename T>
void launch_stencil(const Ctx& c, int ik, const T* Yin, int64_t ld, const T* Yprev, int64_t ld_prev, T* Yout,
                    int64_t ld_out, int ncol, double alpha, double cshift, double beta, hipStream_t st) {
  using RT = typename real_of<T>::type;
  StencilCoef sc;
  fill_stencil_coef(c, ik, sc);
  KArgs<RT> a{};
  for (int p = 0; p <= kMaxR; ++p) {
    a.kx[p] = (RT)sc.kin[0][p];
    a.ky[p] = (RT)sc.kin[1][p];
    a.kz[p] = (RT)sc.kin[2][p];
  }
  a.center = (RT)sc.center;
  a.alpha = (RT)alpha; a.cshift = (RT)cshift; a.beta = (RT)beta;
  for (int d = 0; d < 3; ++d) { a.ph_re[d] = (RT)sc.phase_re[d]; a.ph_im[d] = (RT)sc.phase_im[d]; }
  a.n1 = c.p.n[0]; a.n2 = c.p.n[1]; a.n3 = c.p.n[2];
  a.has_prev = (Yprev != nullptr && beta != 0.0) ? 1 : 0;
  a.ld = ld;
  a.ld_prev = ld_prev;
  a.ld_out = ld_out;
  const StencilShape sh = pick_tiles(c, ncol, (int)sizeof(T));
  const int TX = sh.TX, TYt = sh.TYt, tz = sh.tz;
  const int TY = TYt * sh.RY;
  a.tiles_x = (a.n1 + TX - 1) / TX;
  a.tz = tz;
  dim3 grid(a.tiles_x * ((a.n2 + TY - 1) / TY), (a.n3 + tz - 1) / tz, ncol);
  dim3 block(TX, TYt);
  const int R = sc.R;
  const size_t lds = stencil_lds(a.n1, TX, TYt, sh.RY, R, sh.ring, sizeof(T));
  const bool small = halo_slots(a.n1, TX, TYt, TY, R) <= kHaloSlotsSmall;
  const RT* V;
  if constexpr (sizeof(RT) == 4) V = c.d_Vf; else V = c.d_V;
  const int rg = sh.ring;
  switch (R) {
    case 1: launch_r<T, RT, 1>(sh.RY, small, rg, a, grid, block, lds, Yin, Yprev, Yout, V, st); break;
    case 2: launch_r<T, RT, 2>(sh.RY, small, rg, a, grid, block, lds, Yin, Yprev, Yout, V, st); break;
    case 3: launch_r<T, RT, 3>(sh.RY, small, rg, a, grid, block, lds, Yin, Yprev, Yout, V, st); break;
    case 4: launch_r<T, RT, 4>(sh.RY, small, rg, a, grid, block, lds, Yin, Yprev, Yout, V, st); break;
    case 5: launch_r<T, RT, 5>(sh.RY, small, rg, a, grid, block, lds, Yin, Yprev, Yout, V, st); break;
    default: launch_r<T, RT, 6>(sh.RY, small, rg, a, grid, block, lds, Yin, Yprev, Yout, V, st); break;
  }
}

template <typename T, typename RT, int R>
static void launch_batch_r(int RY, bool small_halo, int ring, dim3 grid, dim3 block, size_t lds,
                           const SJob<RT>* jobs, int njobs, unsigned long long total, unsigned long long* counters,
                           hipStream_t st) {
  if constexpr (R == kRingR) {
    if (ring && counters) {
      auto go = [&](auto kernel) {
        allow_lds(kernel, lds);
        launch_k(kernel, grid, block, lds, st, jobs, njobs, total, counters);
      };
      if (RY == 4) go(k_stencil_batch<T, RT, R, 4, kHaloSlotsSmall, true>);
      else if (RY == 2) go(k_stencil_batch<T, RT, R, 2, kHaloSlotsSmall, true>);
      else go(k_stencil_batch<T, RT, R, 1, kHaloSlotsSmall, true>);
      return;
    }
  }
  if (!counters) {   // one workgroup per item
    dim3 g((unsigned)total);
    if (RY == 4)
      launch_k(k_stencil_multi<T, RT, R, 4>, g, block, lds, st, jobs, njobs);
    else if (RY == 2)
      launch_k(k_stencil_multi<T, RT, R, 2>, g, block, lds, st, jobs, njobs);
    else
      launch_k(k_stencil_multi<T, RT, R, 1>, g, block, lds, st, jobs, njobs);
    return;
  }
  auto go = [&](auto nhs) {
    constexpr int NHS = decltype(nhs)::value;
    if (RY == 4)
      launch_k(k_stencil_batch<T, RT, R, 4, NHS>, grid, block, lds, st, jobs, njobs, total, counters);
    else if (RY == 2)
      launch_k(k_stencil_batch<T, RT, R, 2, NHS>, grid, block, lds, st, jobs, njobs, total, counters);
    else
      launch_k(k_stencil_batch<T, RT, R, 1, NHS>, grid, block, lds, st, jobs, njobs, total, counters);
  };
  if (small_halo) go(std::integral_constant<int, kHaloSlotsSmall>());
  else go(std::integral_constant<int, kHaloSlots>());
}

// Common tile shape for a set of grids: the autotuned shape of the first
// context if every grid admits it, else the largest admissible built-in one.
bool batch_shape(const std::vector<const Ctx*>& cs, int ncol, int elem, int& TX, int& TYt, int& RY, int* TZ,
                 int* ring) {
  const Ctx& c0 = *cs[0];
  StencilShape sh = pick_tiles(c0, ncol, elem);
  auto ok_all = [&](const StencilShape& t) {
    if (t.TX * t.TYt > 512) return false;   // the persistent kernel is built for 512 threads
    for (const Ctx* c : cs)
      if (!shape_ok(*c, StencilShape{t.TX, t.TYt, t.RY, 1, t.ring}, c->p.n0)) return false;
    return true;
  };
  if (!ok_all(sh)) {
    int n1min = 1 << 30, n2min = 1 << 30;
    for (const Ctx* c : cs) { n1min = std::min(n1min, c->p.n[0]); n2min = std::min(n2min, c->p.n[1]); }
    bool found = false;
    for (int ry : {elem > 8 ? 2 : 4, 2, 1}) {
      for (int tx : {std::min(n1min, 128), 64, 32, 16}) {
        if (tx > n1min) continue;
        for (int tyt = std::max(1, 256 / tx); tyt >= 1 && !found; --tyt) {
          StencilShape t{tx, tyt, ry, 1};
          if (tyt * ry <= n2min && ok_all(t)) { sh = t; found = true; }
        }
        if (found) break;
      }
      if (found) break;
    }
    if (!found) return false;
  }
  TX = sh.TX; TYt = sh.TYt; RY = sh.RY;
  if (TZ) *TZ = sh.tz;
  if (ring) *ring = sh.ring;
  return true;
}

// One stencil step for many blocks: the blocks are grouped by the tile shape
// their own grid prefers (tuned or built-in, at most 512 threads, the job's
// own z chunk), each group becoming one persistent launch.
template <typename T>
hcu_status plan_stencil_batch(const std::vector<StencilJob>& jobs, std::vector<unsigned char>& host,
                              std::vector<BatchLaunch>& out) {
  using RT = typename real_of<T>::type;
  if (jobs.empty()) return HCU_OK;
  const int R = jobs[0].c->p.n0;
  for (const StencilJob& j : jobs)
    if (j.c->p.n0 != R) return HCU_INVALID_ARG;
  std::vector<StencilShape> shp(jobs.size());
  std::vector<int> gid(jobs.size());
  std::vector<StencilShape> groups;
  for (size_t i = 0; i < jobs.size(); ++i) {
    int TX, TYt, RY, TZ = 0, ring = 0;
    std::vector<const Ctx*> one{jobs[i].c};
    if (!batch_shape(one, jobs[i].ncol, (int)sizeof(T), TX, TYt, RY, &TZ, &ring)) return HCU_INVALID_ARG;
    shp[i] = StencilShape{TX, TYt, RY, TZ, ring};
    int g = -1;
    for (size_t k = 0; k < groups.size(); ++k)
      if (groups[k].TX == TX && groups[k].TYt == TYt && groups[k].RY == RY && groups[k].ring == ring) g = (int)k;
    if (g < 0) {
      g = (int)groups.size();
      groups.push_back(shp[i]);
    }
    gid[i] = g;
  }
  size_t slot = host.size() / sizeof(SJob<RT>);
  host.resize(host.size() + jobs.size() * sizeof(SJob<RT>), 0);
  SJob<RT>* hj = reinterpret_cast<SJob<RT>*>(host.data());
  for (size_t g = 0; g < groups.size(); ++g) {
    const int TX = groups[g].TX, TYt = groups[g].TYt, RY = groups[g].RY;
    const int TY = TYt * RY;
    BatchLaunch L{slot, 0, 0, TX, TYt, RY, R, 0, groups[g].ring, 0};
    for (size_t i = 0; i < jobs.size(); ++i) {
      if (gid[i] != (int)g) continue;
      const StencilJob& j = jobs[i];
      const Ctx& c = *j.c;
      L.halo_slots = std::max(L.halo_slots, halo_slots(c.p.n[0], TX, TYt, TY, R));
      L.halo_n = std::max(L.halo_n, halo_values(c.p.n[0], TX, TY, R));
      StencilCoef sc;
      fill_stencil_coef(c, j.ik, sc);
      KArgs<RT> a{};
      for (int p = 0; p <= kMaxR; ++p) {
        a.kx[p] = (RT)sc.kin[0][p];
        a.ky[p] = (RT)sc.kin[1][p];
        a.kz[p] = (RT)sc.kin[2][p];
      }
      a.center = (RT)sc.center;
      a.alpha = (RT)j.alpha; a.cshift = (RT)j.cshift; a.beta = (RT)j.beta;
      for (int d = 0; d < 3; ++d) { a.ph_re[d] = (RT)sc.phase_re[d]; a.ph_im[d] = (RT)sc.phase_im[d]; }
      a.n1 = c.p.n[0]; a.n2 = c.p.n[1]; a.n3 = c.p.n[2];
      a.has_prev = (j.Yprev != nullptr && j.beta != 0.0) ? 1 : 0;
      a.ld = j.ld; a.ld_prev = j.ld_prev; a.ld_out = j.ld_out;
      a.tiles_x = (a.n1 + TX - 1) / TX;
      const int tiles = a.tiles_x * ((a.n2 + TY - 1) / TY);
      // the job's own z chunk (tuned or built-in); the fallback shape has none
      a.tz = shp[i].tz > 1 ? std::min(a.n3, shp[i].tz) : std::max(8, std::min(a.n3, 24));
      const int nzc = (a.n3 + a.tz - 1) / a.tz;
      SJob<RT>& h = hj[slot++];
      h.Yin = j.Yin; h.Yprev = j.Yprev; h.Yout = j.Yout;
      if constexpr (sizeof(RT) == 4) h.V = c.d_Vf; else h.V = c.d_V;
      h.a = a;
      h.ntiles = tiles;
      h.nzc = nzc;
      h.item_begin = L.total;
      L.total += (unsigned long long)tiles * nzc * j.ncol;
      ++L.njob;
    }
    out.push_back(L);
  }
  return HCU_OK;
}

template <typename T>
hcu_status run_stencil_batch(const BatchLaunch& L, const void* d_jobs, unsigned long long* d_counters,
                             hipStream_t st) {
  using RT = typename real_of<T>::type;
  if (d_counters && hipMemsetAsync(d_counters, 0, kNumXcd * sizeof(unsigned long long), st) != hipSuccess)
    return HCU_DEVICE;
  size_t lds = stencil_lds(0, L.TX, L.TYt, L.RY, L.R, 0, sizeof(T));
  if (L.ring) lds += (size_t)L.R * L.halo_n * sizeof(T);
  const bool small = L.halo_slots <= kHaloSlotsSmall;
  dim3 grid(1024), block(L.TX, L.TYt);
  const SJob<RT>* dj = reinterpret_cast<const SJob<RT>*>(d_jobs) + L.first;
  switch (L.R) {
    case 1:
      launch_batch_r<T, RT, 1>(L.RY, small, L.ring, grid, block, lds, dj, L.njob, L.total, d_counters, st);
      break;
    case 2:
      launch_batch_r<T, RT, 2>(L.RY, small, L.ring, grid, block, lds, dj, L.njob, L.total, d_counters, st);
      break;
    case 3:
      launch_batch_r<T, RT, 3>(L.RY, small, L.ring, grid, block, lds, dj, L.njob, L.total, d_counters, st);
      break;
    case 4:
      launch_batch_r<T, RT, 4>(L.RY, small, L.ring, grid, block, lds, dj, L.njob, L.total, d_counters, st);
      break;
    case 5:
      launch_batch_r<T, RT, 5>(L.RY, small, L.ring, grid, block, lds, dj, L.njob, L.total, d_counters, st);
      break;
    default:
      launch_batch_r<T, RT, 6>(L.RY, small, L.ring, grid, block, lds, dj, L.njob, L.total, d_counters, st);
      break;
  }
  return hipGetLastError() == hipSuccess ? HCU_OK : HCU_DEVICE;
}

#define INST_STENCIL(T)                                                                                 \
  template void launch_stencil<T>(const Ctx&, int, const T*, int64_t, const T*, int64_t, T*, int64_t, int, \
                                  double, double, double, hipStream_t);                                \
  template hcu_status plan_stencil_batch<T>(const std::vector<StencilJob>&, std::vector<unsigned char>&,   \
                                            std::vector<BatchLaunch>&);                                    \
  template hcu_status run_stencil_batch<T>(const BatchLaunch&, const void*, unsigned long long*, hipStream_t);
INST_STENCIL(double)
INST_STENCIL(float)
INST_STENCIL(cplx<double>)
INST_STENCIL(cplx<float>)

}  // namespace hcu
