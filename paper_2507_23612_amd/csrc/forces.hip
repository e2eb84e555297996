// Hubbard atomic forces and Hubbard stress tensor (Sec. II.A: the force
// section, Eq. Force1 -> Eq. DerR -> the final force expression; the stress
// section, Eq. StressDef -> the final stress expression).  As the paper does
// for the finite-difference method, the derivative of each atomic orbital is
// moved to the Kohn-Sham orbitals and taken with the centred gradient stencil
// whose weights it prints (Sec. II.B):
//
//   P_mj = <phi_m|psi_j> dV,  G^a_mj = <phi_m|d_a psi_j> dV,
//   Q^ab_mj = <phi^b_m|d_a psi_j> dV,  phi^b(x) = sum_T phi(x-R-T)(x-R-T)_b e^{ik.T},
//   f^J_a     = g sum_k w_k Re sum_mm' U (2 D_m'm - delta_mm') sum_j f_j P_mj conj(G^a_m'j)
//   sigma_ab  = g/|Omega| sum_I sum_mm' U/2 (delta_mm' - 2 D_m'm)
//               [-2 sum_k w_k Re sum_j f_j Q^ab_mj conj(P_m'j) - delta_ab D_mm']
//
// with g = 2 for spin-unpolarised runs (both channels carry the stored D, as
// in E_U) and D the occupation matrix of the orbitals and occupations used.
// The printed expressions carry D_mm' in the first factor; it equals D_m'm
// for the real D of the Gamma point and of k-sets closed under k -> -k, and
// D_m'm is the exact derivative of E_U for complex D as well.
//
// Device work per (spin, k): the three gradient blocks (the context's work
// blocks), the projections of X and of the gradients onto the orbitals and
// onto their moment functions (the projection-brick kernels, with the
// moment functions evaluated into tables of the same layout), and one small
// kernel per Hubbard atom that forms the occupation-weighted bilinear sums;
// the host combines them over k-points and spins.
#include "common.h"

#include <cmath>
#include <complex>
#include <cstring>

namespace hcu {

struct GradCoef {
  int n[3];
  int R;
  double w[3][kMaxR];   // printed gradient weights per axis, p = 1..R
  double theta[3];      // k_a L_a: phase of one wrap around axis a
};

// Gradient of every state of X along the three axes (Sec. II.B stencil):
// sum_p w_p (f(i+p) - f(i-p)), indices outside the cell mapped back with
// the Bloch factor of each wrap.  One thread per (point, state), consecutive
// threads along x, so every neighbour load is coalesced.
template <typename T>
__global__ __launch_bounds__(256) void k_grad3(const T* __restrict__ X, int64_t ld, T* __restrict__ G0,
                                               T* __restrict__ G1, T* __restrict__ G2, int64_t ldg, GradCoef gc) {
  using R = typename real_of<T>::type;
  const int64_t nd = (int64_t)gc.n[0] * gc.n[1] * gc.n[2];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nd) return;
  const int s = blockIdx.y;
  const T* __restrict__ x = X + (int64_t)s * ld;
  const int ci[3] = {(int)(p % gc.n[0]), (int)((p / gc.n[0]) % gc.n[1]), (int)(p / ((int64_t)gc.n[0] * gc.n[1]))};
  const int64_t stride[3] = {1, (int64_t)gc.n[0], (int64_t)gc.n[0] * gc.n[1]};
  T* out[3] = {G0, G1, G2};
  for (int a = 0; a < 3; ++a) {
    const int na = gc.n[a];
    T acc = T(0);
    for (int q = 1; q <= gc.R; ++q) {
      int ip = ci[a] + q, wp = 0;
      while (ip >= na) { ip -= na; ++wp; }
      int im = ci[a] - q, wm = 0;
      while (im < 0) { im += na; --wm; }
      T fp = x[p + (int64_t)(ip - ci[a]) * stride[a]];
      T fm = x[p + (int64_t)(im - ci[a]) * stride[a]];
      if constexpr (sizeof(T) != sizeof(R)) {
        if (wp) fp = fp * T((R)cos(wp * gc.theta[a]), (R)sin(wp * gc.theta[a]));
        if (wm) fm = fm * T((R)cos(wm * gc.theta[a]), (R)sin(wm * gc.theta[a]));
      }
      acc += (R)gc.w[a][q - 1] * (fp - fm);
    }
    out[a][(int64_t)s * ldg + p] = acc;
  }
}

constexpr int kBilin = 325;   // 25 (D) + 3 x 25 (forces) + 9 x 25 (stress) complex sums per atom

// Bilinear sums of one Hubbard atom (one workgroup), summed over the states
// in a fixed order: thread t forms sum_s f_s X_{m s} conj(Y_{m' s}) for
//   t <  25 : X = P,      Y = P        (occupation matrix of this (spin, k))
//   t < 100 : X = P,      Y = G^a      (forces, a = (t - 25) / 25)
//   t < 325 : X = Q^ab,   Y = P        (stress, 3a + b = (t - 100) / 25)
// proj holds 13 arrays [ns][nproj] at multiples of pstride: P, G^0..2,
// Q^{ab} at 4 + 3a + b.
template <typename T>
__global__ __launch_bounds__(384) void k_hub_bilinear(const T* __restrict__ proj, int64_t pstride, int ns, int nproj,
                                                      const double* __restrict__ occ,
                                                      const BlockDesc* __restrict__ blocks,
                                                      const int* __restrict__ hub_blocks, int nsum,
                                                      double* __restrict__ out) {
  using R = typename real_of<T>::type;
  const BlockDesc b = blocks[hub_blocks[blockIdx.x]];
  const int t = threadIdx.x;
  if (t >= kBilin) return;
  int xi, yi, e;
  if (t < 25) { xi = 0; yi = 0; e = t; }
  else if (t < 100) { xi = 0; yi = 1 + (t - 25) / 25; e = (t - 25) % 25; }
  else { xi = 4 + (t - 100) / 25; yi = 0; e = (t - 100) % 25; }
  const int m = e / 5, mp = e % 5;
  double re = 0, im = 0;
  if (t < nsum && m < b.nm && mp < b.nm) {
    const T* __restrict__ X = proj + xi * pstride + b.j0 + m;
    const T* __restrict__ Y = proj + yi * pstride + b.j0 + mp;
    for (int s = 0; s < ns; ++s) {
      const T v = mul_conj(X[(int64_t)s * nproj], Y[(int64_t)s * nproj]);
      const double f = occ[s];
      if constexpr (sizeof(T) == sizeof(R)) {
        re += f * (double)v;
      } else {
        re += f * (double)v.re;
        im += f * (double)v.im;
      }
    }
  }
  double* o = out + 2 * ((size_t)b.hub * kBilin + t);
  o[0] = re;
  o[1] = im;
}

template <typename T>
hcu_status forces_stress_t(Ctx& c, const double* occ_host, double* forces, double* stress) {
  const int nh = (int)c.hub_atoms.size();
  const int ns = c.p.ns, nsk = c.p.nspin * c.p.nk;
  const int64_t nd = c.nd;
  hipStream_t st = c.stream;
  if (forces) std::memset(forces, 0, sizeof(double) * 3 * c.p.natom);
  if (stress) std::memset(stress, 0, sizeof(double) * 9);
  if (nh == 0) return HCU_OK;
  const double* occ = c.d_occ;
  if (occ_host) {
    for (int i = 0; i < nsk * ns; ++i)
      if (!std::isfinite(occ_host[i])) return HCU_NAN;
    HCU_HIP(hipMemcpyAsync(c.d_focc, occ_host, sizeof(double) * nsk * ns, hipMemcpyHostToDevice, st));
    occ = c.d_focc;
  }
  const bool want_stress = stress != nullptr;
  const int nsum = want_stress ? kBilin : 100;
  // printed gradient weights (Sec. II.B): (-1)^(p+1) / (h p) (n0!)^2 / ((n0-p)! (n0+p)!)
  GradCoef gc{};
  const int R = c.p.n0;
  gc.R = R;
  for (int a = 0; a < 3; ++a) {
    gc.n[a] = c.p.n[a];
    for (int p = 1; p <= R; ++p) {
      double bin = 1.0;   // (n0!)^2 / ((n0-p)!(n0+p)!) = prod_{i=1..p} (n0-p+i)/(n0+i)
      for (int i = 1; i <= p; ++i) bin *= (double)(R - p + i) / (double)(R + i);
      gc.w[a][p - 1] = ((p % 2) ? 1.0 : -1.0) / (c.h[a] * p) * bin;
    }
  }
  std::vector<double> sums((size_t)nsk * nh * kBilin * 2, 0.0);
  const int64_t pstride = (int64_t)ns * c.nproj;
  T* PR = (T*)c.d_fproj;
  for (int ik = 0; ik < c.p.nk; ++ik) {
    if (want_stress)
      for (int b = 0; b < 3; ++b) {
        hcu_status s = build_moment_table<T>(c, ik, b, (T*)c.d_momcsc, (T*)c.d_mom[b], st);
        if (s != HCU_OK) return s;
      }
    for (int a = 0; a < 3; ++a) gc.theta[a] = c.kpts[3 * ik + a] * c.p.L[a];
    for (int spin = 0; spin < c.p.nspin; ++spin) {
      const int sk = sk_index(c, spin, ik);
      const T* X = (const T*)c.d_X[sk];
      T* Gr[3] = {(T*)c.d_W[3 * sk], (T*)c.d_W[3 * sk + 1], (T*)c.d_W[3 * sk + 2]};
      launch_k(k_grad3<T>, dim3((unsigned)((nd + 255) / 256), ns), 256, 0, st, X, nd, Gr[0], Gr[1], Gr[2], nd, gc);
      const T* tab = (const T*)c.d_pbval[ik];
      launch_project_table<T>(c, tab, X, ns, nd, PR, st);
      for (int a = 0; a < 3; ++a) launch_project_table<T>(c, tab, Gr[a], ns, nd, PR + (1 + a) * pstride, st);
      if (want_stress)
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b)
            launch_project_table<T>(c, (const T*)c.d_mom[b], Gr[a], ns, nd, PR + (4 + 3 * a + b) * pstride, st);
      launch_k(k_hub_bilinear<T>, nh, 384, 0, st, (const T*)PR, pstride, ns, c.nproj, occ + (size_t)sk * ns,
               c.d_blocks, c.d_hub_blocks, nsum, c.d_fsum);
      HCU_HIP(hipGetLastError());
      HCU_HIP(hipMemcpyAsync(sums.data() + (size_t)sk * nh * kBilin * 2, c.d_fsum,
                             sizeof(double) * nh * kBilin * 2, hipMemcpyDeviceToHost, st));
    }
  }
  HCU_HIP(hipStreamSynchronize(st));
  // combine over k-points and spins (host, FP64)
  using Z = std::complex<double>;
  const double g = c.p.nspin == 1 ? 2.0 : 1.0;
  const double omega = c.p.L[0] * c.p.L[1] * c.p.L[2];
  auto at = [&](int sk, int h, int t) {
    const double* v = sums.data() + 2 * (((size_t)sk * nh + h) * kBilin + t);
    return Z(v[0], v[1]);
  };
  for (int spin = 0; spin < c.p.nspin; ++spin)
    for (int h = 0; h < nh; ++h) {
      const int nm = 2 * c.hub_l[h] + 1;
      const double U = c.hub_U[h];
      Z D[25];
      for (int e = 0; e < 25; ++e) {
        D[e] = 0;
        for (int ik = 0; ik < c.p.nk; ++ik) D[e] += c.kw[ik] * at(sk_index(c, spin, ik), h, e);
      }
      // W = U (2 D^T - 1) (= -2 dE_U/dD),  V = U/2 (1 - 2 D^T) (= dE_U/dD)
      Z W[25], V[25];
      for (int m = 0; m < nm; ++m)
        for (int mp = 0; mp < nm; ++mp) {
          const double d = m == mp ? 1.0 : 0.0;
          W[m * 5 + mp] = U * (2.0 * D[mp * 5 + m] - d);
          V[m * 5 + mp] = 0.5 * U * (d - 2.0 * D[mp * 5 + m]);
        }
      const int atom = c.hub_atoms[h];
      for (int ik = 0; ik < c.p.nk; ++ik) {
        const int sk = sk_index(c, spin, ik);
        for (int a = 0; a < 3; ++a) {
          if (forces) {
            Z acc = 0;
            for (int m = 0; m < nm; ++m)
              for (int mp = 0; mp < nm; ++mp) acc += W[m * 5 + mp] * at(sk, h, 25 + 25 * a + m * 5 + mp);
            forces[3 * atom + a] += g * c.kw[ik] * acc.real();
          }
          if (stress)
            for (int b = 0; b < 3; ++b) {
              Z acc = 0;
              for (int m = 0; m < nm; ++m)
                for (int mp = 0; mp < nm; ++mp)
                  acc += V[m * 5 + mp] * at(sk, h, 100 + 25 * (3 * a + b) + m * 5 + mp);
              stress[3 * a + b] += g / omega * c.kw[ik] * (-2.0) * acc.real();
            }
        }
      }
      if (stress) {
        Z tr = 0;
        for (int m = 0; m < nm; ++m)
          for (int mp = 0; mp < nm; ++mp) tr += V[m * 5 + mp] * D[m * 5 + mp];
        for (int a = 0; a < 3; ++a) stress[4 * a] -= g / omega * tr.real();
      }
    }
  for (int i = 0; forces && i < 3 * c.p.natom; ++i)
    if (!std::isfinite(forces[i])) return HCU_NAN;
  for (int i = 0; stress && i < 9; ++i)
    if (!std::isfinite(stress[i])) return HCU_NAN;
  return HCU_OK;
}

hcu_status hubbard_forces_stress(Ctx& c, const double* occ, double* forces, double* stress) {
  if (c.any_complex) {
    return c.mixed ? forces_stress_t<cplx<float>>(c, occ, forces, stress)
                   : forces_stress_t<cplx<double>>(c, occ, forces, stress);
  }
  return c.mixed ? forces_stress_t<float>(c, occ, forces, stress) : forces_stress_t<double>(c, occ, forces, stress);
}

}  // namespace hcu
