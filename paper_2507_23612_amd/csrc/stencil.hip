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

namespace hcu {

// points per thread along y: fewer for double complex to bound registers
template <typename T> constexpr int ry_of() { return sizeof(T) > 8 ? 2 : 4; }

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

template <typename T> struct Ld {
  // value of the (possibly wrapped) node with wrap counts w (each -1, 0, 1)
  template <typename RT>
  __device__ static inline T get(const T* __restrict__ y, int64_t idx, int wx, int wy, int wz, const KArgs<RT>&) {
    (void)wx; (void)wy; (void)wz;
    return y[idx];
  }
};
template <typename R> struct Ld<cplx<R>> {
  template <typename RT>
  __device__ static inline cplx<R> get(const cplx<R>* __restrict__ y, int64_t idx, int wx, int wy, int wz,
                                       const KArgs<RT>& a) {
    cplx<R> v = y[idx];
    int w[3] = {wx, wy, wz};
    for (int d = 0; d < 3; ++d) {
      if (w[d] == 0) continue;
      cplx<R> ph(a.ph_re[d], w[d] > 0 ? a.ph_im[d] : -a.ph_im[d]);
      for (int t = 0; t < (w[d] > 0 ? w[d] : -w[d]); ++t) v = v * ph;
    }
    return v;
  }
};

// periodic image of grid coordinate g: returns g - w n in [0, n), w = floor(g / n)
__device__ inline int wrap(int g, int n, int& w) {
  w = (g >= 0) ? g / n : -((n - 1 - g) / n);
  return g - w * n;
}

template <typename T, typename RT, int R, int RY>
__global__ __launch_bounds__(256) void k_stencil(const T* __restrict__ Yin, const T* __restrict__ Yprev,
                                                 T* __restrict__ Yout, const RT* __restrict__ V,
                                                 const KArgs<RT> a) {
  extern __shared__ unsigned char smem_raw[];
  T* sp = reinterpret_cast<T*>(smem_raw);
  const int TX = blockDim.x, TYt = blockDim.y, TY = TYt * RY;
  const int SW = TX + 2 * R;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int tid = ty * TX + tx, nthr = TX * TYt;
  const int bx = blockIdx.x % a.tiles_x, by = blockIdx.x / a.tiles_x;
  const int x0 = bx * TX, y0 = by * TY;
  const int zbeg = blockIdx.y * a.tz;
  const int zend = min(zbeg + a.tz, a.n3);
  const int64_t s = blockIdx.z;
  const T* __restrict__ Ys = Yin + s * a.ld;
  const int n1 = a.n1, n2 = a.n2, n3 = a.n3;
  const int64_t plane = (int64_t)n1 * n2;

  int wxo, wyo[RY];
  const int gx = wrap(x0 + tx, n1, wxo);      // wxo == 1 only for ragged tiles
  int gy[RY];
  for (int r = 0; r < RY; ++r) gy[r] = wrap(y0 + ty * RY + r, n2, wyo[r]);

  T q[RY][2 * R + 1];
  // prime the z queue with planes zbeg-R .. zbeg+R-1
  for (int dz = -R; dz < R; ++dz) {
    int wz;
    int gz = wrap(zbeg + dz, n3, wz);
    for (int r = 0; r < RY; ++r)
      q[r][dz + R] = Ld<T>::get(Ys, gx + (int64_t)n1 * gy[r] + plane * gz, wxo, wyo[r], wz, a);
  }

  for (int z = zbeg; z < zend; ++z) {
    {
      int wz;
      int gz = wrap(z + R, n3, wz);
      for (int r = 0; r < RY; ++r)
        q[r][2 * R] = Ld<T>::get(Ys, gx + (int64_t)n1 * gy[r] + plane * gz, wxo, wyo[r], wz, a);
    }
    __syncthreads();
    for (int r = 0; r < RY; ++r) sp[(ty * RY + r + R) * SW + tx + R] = q[r][R];
    const int64_t zoff = plane * z;
    // x halo: TY rows x 2R columns
    for (int e = tid; e < TY * 2 * R; e += nthr) {
      int row = e / (2 * R), cc = e % (2 * R);
      int col = cc < R ? cc : TX + cc;
      int wx, wy;
      int hx = wrap(x0 + col - R, n1, wx);
      int hy = wrap(y0 + row, n2, wy);
      sp[(row + R) * SW + col] = Ld<T>::get(Ys, hx + (int64_t)n1 * hy + zoff, wx, wy, 0, a);
    }
    // y halo: 2R rows x TX columns
    for (int e = tid; e < 2 * R * TX; e += nthr) {
      int rh = e / TX, col = e % TX;
      int row = rh < R ? rh : TY + rh;
      int wx, wy;
      int hx = wrap(x0 + col, n1, wx);
      int hy = wrap(y0 + row - R, n2, wy);
      sp[row * SW + col + R] = Ld<T>::get(Ys, hx + (int64_t)n1 * hy + zoff, wx, wy, 0, a);
    }
    __syncthreads();

    T strip[RY + 2 * R];
    for (int t = 0; t < RY + 2 * R; ++t) strip[t] = sp[(ty * RY + t) * SW + tx + R];
    for (int r = 0; r < RY; ++r) {
      const int row = ty * RY + r + R;
      const T* L = sp + row * SW + tx + R;
      T acc = T(0);
      for (int p = 1; p <= R; ++p) {
        acc += a.kx[p] * (L[p] + L[-p]);
        acc += a.ky[p] * (strip[r + R + p] + strip[r + R - p]);
        acc += a.kz[p] * (q[r][R + p] + q[r][R - p]);
      }
      const bool active = (x0 + tx < n1) && (y0 + ty * RY + r < n2);
      if (active) {
        const int64_t pidx = gx + (int64_t)n1 * gy[r] + zoff;
        const T cen = q[r][R];
        acc += (a.center + V[pidx] - a.cshift) * cen;
        T out = a.alpha * acc;
        if (a.has_prev) out += (-a.beta) * Yprev[s * a.ld_prev + pidx];
        Yout[s * a.ld_out + pidx] = out;
      }
    }
    for (int r = 0; r < RY; ++r)
      for (int t = 0; t < 2 * R; ++t) q[r][t] = q[r][t + 1];
  }
}

// Tile shape for a grid (TX threads along x, TYt thread rows, RY points each).
static void pick_tiles(const Ctx& c, int RY, int& TX, int& TYt, int& tz, int ncol) {
  const int n1 = c.p.n[0], n2 = c.p.n[1], n3 = c.p.n[2];
  if (c.tile_x > 0) {
    TX = c.tile_x; TYt = c.tile_yt; tz = c.tile_z;
  } else {
    TX = n1 <= 128 ? n1 : 64;
    TYt = std::max(1, 256 / TX);
    tz = 0;
  }
  TX = std::min(TX, n1);
  while (TYt > 1 && TYt * RY > n2) --TYt;
  if (TYt * RY > n2) TYt = 1;
  if (tz <= 0) {
    int tiles = ((n1 + TX - 1) / TX) * ((n2 + TYt * RY - 1) / (TYt * RY));
    int zs = 1;
    while ((int64_t)tiles * zs * ncol < 2048 && n3 / (zs * 2) >= 16) zs *= 2;
    tz = (n3 + zs - 1) / zs;
  }
}

template <typename T, typename RT, int R>
static void launch_r(const KArgs<RT>& a, dim3 grid, dim3 block, size_t lds, const T* Yin, const T* Yprev, T* Yout,
                     const RT* V, hipStream_t st) {
  k_stencil<T, RT, R, ry_of<T>()><<<grid, block, lds, st>>>(Yin, Yprev, Yout, V, a);
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
  int TX, TYt, tz;
  pick_tiles(c, ry_of<T>(), TX, TYt, tz, ncol);
  const int TY = TYt * ry_of<T>();
  a.tiles_x = (a.n1 + TX - 1) / TX;
  a.tz = tz;
  dim3 grid(a.tiles_x * ((a.n2 + TY - 1) / TY), (a.n3 + tz - 1) / tz, ncol);
  dim3 block(TX, TYt);
  const int R = sc.R;
  size_t lds = (size_t)(TY + 2 * R) * (TX + 2 * R) * sizeof(T);
  const RT* V;
  if constexpr (sizeof(RT) == 4) V = c.d_Vf; else V = c.d_V;
  switch (R) {
    case 1: launch_r<T, RT, 1>(a, grid, block, lds, Yin, Yprev, Yout, V, st); break;
    case 2: launch_r<T, RT, 2>(a, grid, block, lds, Yin, Yprev, Yout, V, st); break;
    case 3: launch_r<T, RT, 3>(a, grid, block, lds, Yin, Yprev, Yout, V, st); break;
    case 4: launch_r<T, RT, 4>(a, grid, block, lds, Yin, Yprev, Yout, V, st); break;
    case 5: launch_r<T, RT, 5>(a, grid, block, lds, Yin, Yprev, Yout, V, st); break;
    default: launch_r<T, RT, 6>(a, grid, block, lds, Yin, Yprev, Yout, V, st); break;
  }
}

#define INST_STENCIL(T)                                                                                 \
  template void launch_stencil<T>(const Ctx&, int, const T*, int64_t, const T*, int64_t, T*, int64_t, int, \
                                  double, double, double, hipStream_t);
INST_STENCIL(double)
INST_STENCIL(float)
INST_STENCIL(cplx<double>)
INST_STENCIL(cplx<float>)

}  // namespace hcu
