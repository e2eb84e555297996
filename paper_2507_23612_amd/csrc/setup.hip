// Problem setup: per-atom supports and projector blocks (host, integer
// bookkeeping), and on the device: the local potential, the Bloch-mapped
// atom-centred functions on each atom's compact support, the optional per-atom
// Loewdin orthonormalisation and the per-point (CSR) copy of the values.
//
// Paper: atomic orbitals are real spherical harmonics times radial functions,
// truncated where the radial value falls below a threshold and not stored
// beyond it (Sec. II.B); orbitals are Bloch periodically mapped, with image
// phases e^{-i k.(R_I - R_I~)} (Sec. II.A, energy section); DFT+U is handled
// like the nonlocal projectors, all integrals of one atom together
// (Sec. II.B).
#include "common.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace hcu {

// ------------------------------------------------------------------ radials
static double fact(int n) { double f = 1; for (int i = 2; i <= n; ++i) f *= i; return f; }

// N such that int (N r^p e^{-alpha r})^2 r^2 dr = 1
static double hub_norm(int p, double a) { return std::sqrt(std::pow(2 * a, 2 * p + 3) / fact(2 * p + 2)); }
// N such that int (N r^l e^{-r^2/(2w^2)})^2 r^2 dr = 1
static double kb_norm(int l, double w) { return std::sqrt(2.0 / (std::tgamma(l + 1.5) * std::pow(w, 2 * l + 3))); }

__host__ __device__ inline double hub_radial(double r, double N, int p, double a) {
  double rp = 1.0;
  for (int i = 0; i < p; ++i) rp *= r;
  return N * rp * exp(-a * r);
}
__host__ __device__ inline double kb_radial(double r, double N, int l, double w) {
  double rl = (l == 0) ? 1.0 : (l == 1 ? r : r * r);
  return N * rl * exp(-r * r / (2 * w * w));
}

// Outermost radius where f(r) = thr: march inward from 60 bohr in 1e-3
// steps to the first sample >= thr, then bisect the bracketing step.
template <typename F>
static double outer_crossing(F f, double thr) {
  const double step = 1e-3;
  double r = 60.0;
  while (r > 0 && f(r) < thr) r -= step;
  if (r <= 0) return -1.0;
  double lo = r, hi = r + step;   // f(lo) >= thr > f(hi)
  for (int it = 0; it < 200; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    if (f(mid) >= thr) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

// Real spherical harmonics, l <= 2, m = -l..l (orthonormal on the sphere):
// l=1: sqrt(3/4pi) (y, z, x)/r; l=2: sqrt(15/4pi) xy, yz, sqrt(5/16pi)(3z^2-r^2),
// sqrt(15/4pi) xz, sqrt(15/16pi)(x^2-y^2), over r^2.  Zero at r = 0 (l > 0).
__host__ __device__ inline void real_ylm(int l, double x, double y, double z, double* out) {
  const double pi = 3.14159265358979323846;
  double r2 = x * x + y * y + z * z;
  if (l == 0) { out[0] = 0.5 / sqrt(pi); return; }
  if (r2 == 0.0) { for (int m = 0; m < 2 * l + 1; ++m) out[m] = 0.0; return; }
  if (l == 1) {
    double c = sqrt(3.0 / (4 * pi)) / sqrt(r2);
    out[0] = c * y; out[1] = c * z; out[2] = c * x;
    return;
  }
  double c1 = sqrt(15.0 / (4 * pi)) / r2, c0 = sqrt(5.0 / (16 * pi)) / r2, c2 = sqrt(15.0 / (16 * pi)) / r2;
  out[0] = c1 * x * y; out[1] = c1 * y * z; out[2] = c0 * (3 * z * z - r2);
  out[3] = c1 * x * z; out[4] = c2 * (x * x - y * y);
}

// ------------------------------------------------------------------ host structure
static void support_of(const Ctx& c, const double* R, double rc, std::vector<int>& out) {
  const int* n = c.p.n;
  const double* L = c.p.L;
  int nim[3];
  for (int a = 0; a < 3; ++a) nim[a] = (int)std::ceil(rc / L[a]) + 1;
  std::vector<int> pts;
  for (int t3 = -nim[2]; t3 <= nim[2]; ++t3)
    for (int t2 = -nim[1]; t2 <= nim[1]; ++t2)
      for (int t1 = -nim[0]; t1 <= nim[0]; ++t1) {
        double cc[3] = {R[0] + t1 * L[0], R[1] + t2 * L[1], R[2] + t3 * L[2]};
        int lo[3], hi[3];
        bool empty = false;
        for (int a = 0; a < 3; ++a) {
          lo[a] = std::max((int)std::ceil((cc[a] - rc) / c.h[a]), 0);
          hi[a] = std::min((int)std::floor((cc[a] + rc) / c.h[a]), n[a] - 1);
          if (lo[a] > hi[a]) empty = true;
        }
        if (empty) continue;
        for (int k = lo[2]; k <= hi[2]; ++k)
          for (int j = lo[1]; j <= hi[1]; ++j)
            for (int i = lo[0]; i <= hi[0]; ++i) {
              double dx = i * c.h[0] - cc[0], dy = j * c.h[1] - cc[1], dz = k * c.h[2] - cc[2];
              double r = std::sqrt(dx * dx + dy * dy + dz * dz);
              if (r <= rc) pts.push_back(i + n[0] * (j + n[1] * k));
            }
      }
  std::sort(pts.begin(), pts.end());
  pts.erase(std::unique(pts.begin(), pts.end()), pts.end());
  out.swap(pts);
}

hcu_status build_structure(Ctx& c) {
  const hcu_problem& p = c.p;
  c.blocks.clear();
  c.supp.clear();
  c.hub_atoms.clear();
  c.hub_l.clear();
  c.hub_U.clear();
  int j0 = 0, coup = 0;
  int64_t voff = 0;
  std::vector<int> sp;
  for (int ia = 0; ia < p.natom; ++ia) {
    const hcu_species& s = c.species[c.atom_species[ia]];
    const double* R = &c.pos[3 * ia];
    if (s.n_kb > 0) {
      BlockDesc b{};
      b.atom = ia; b.type = 0; b.hub = -1;
      b.nchan = s.n_kb;
      b.width = s.kb_width;
      double rmax = 0;
      int nm = 0;
      for (int ch = 0; ch < s.n_kb; ++ch) {
        int l = s.kb_l[ch];
        double N = kb_norm(l, s.kb_width);
        double rc = outer_crossing([&](double r) { return kb_radial(r, N, l, s.kb_width); }, s.threshold);
        if (rc <= 0) { c.err = "KB radial function never reaches the threshold"; return HCU_INVALID_ARG; }
        b.chan_l[ch] = l; b.chan_rc[ch] = rc; b.chan_norm[ch] = N; b.chan_gamma[ch] = s.kb_gamma[ch];
        rmax = std::max(rmax, rc);
        nm += 2 * l + 1;
      }
      if (nm > kMaxNm) { c.err = "too many KB functions per atom (max 9)"; return HCU_INVALID_ARG; }
      b.nm = nm;
      for (int a = 0; a < 3; ++a) b.center[a] = R[a];
      support_of(c, R, rmax, sp);
      b.nsupp = (int)sp.size();
      b.supp_off = (int64_t)c.supp.size();
      c.supp.insert(c.supp.end(), sp.begin(), sp.end());
      b.val_off = voff; voff += (int64_t)nm * b.nsupp;
      b.j0 = j0; j0 += nm;
      b.coup_off = coup; coup += nm * nm;
      c.blocks.push_back(b);
    }
    if (s.hub_l >= 0) {
      BlockDesc b{};
      b.atom = ia; b.type = 1; b.hub = (int)c.hub_atoms.size();
      int l = s.hub_l;
      b.nchan = 1;
      b.power = s.hub_power; b.alpha = s.hub_alpha;
      double N = hub_norm(s.hub_power, s.hub_alpha);
      double rc = outer_crossing([&](double r) { return hub_radial(r, N, s.hub_power, s.hub_alpha); }, s.threshold);
      if (rc <= 0) { c.err = "Hubbard radial function never reaches the threshold"; return HCU_INVALID_ARG; }
      b.chan_l[0] = l; b.chan_rc[0] = rc; b.chan_norm[0] = N; b.chan_gamma[0] = 0;
      b.nm = 2 * l + 1;
      for (int a = 0; a < 3; ++a) b.center[a] = R[a];
      support_of(c, R, rc, sp);
      b.nsupp = (int)sp.size();
      b.supp_off = (int64_t)c.supp.size();
      c.supp.insert(c.supp.end(), sp.begin(), sp.end());
      b.val_off = voff; voff += (int64_t)b.nm * b.nsupp;
      b.j0 = j0; j0 += b.nm;
      b.coup_off = coup; coup += b.nm * b.nm;
      c.blocks.push_back(b);
      c.hub_atoms.push_back(ia);
      c.hub_l.push_back(l);
      c.hub_U.push_back(s.hub_U);
    }
  }
  c.nproj = j0;
  c.nval = voff;
  c.coup_size = coup;
  // per-point (CSR) view of the same functions, columns ascending
  c.csr_ptr.assign(c.nd + 1, 0);
  for (const BlockDesc& b : c.blocks)
    for (int q = 0; q < b.nsupp; ++q) c.csr_ptr[c.supp[b.supp_off + q] + 1] += b.nm;
  for (int i = 0; i < c.nd; ++i) c.csr_ptr[i + 1] += c.csr_ptr[i];
  const int64_t nnz = c.csr_ptr[c.nd];
  c.csr_col.assign(nnz, 0);
  c.csr_src.assign(nnz, 0);
  std::vector<int> fill(c.csr_ptr.begin(), c.csr_ptr.end() - 1);
  for (const BlockDesc& b : c.blocks)
    for (int m = 0; m < b.nm; ++m)
      for (int q = 0; q < b.nsupp; ++q) {
        int pt = c.supp[b.supp_off + q];
        int e = fill[pt]++;
        c.csr_col[e] = b.j0 + m;
        c.csr_src[e] = b.val_off + (int64_t)m * b.nsupp + q;
      }
  // (the per-point rows are sorted below)
  // within a row, order by column (blocks were visited in order, m inner to
  // the block, but all m of one block precede the next block: already sorted
  // except that rows interleave m-major fills of one block; sort to be safe)
  for (int i = 0; i < c.nd; ++i) {
    int a = c.csr_ptr[i], e = c.csr_ptr[i + 1];
    std::vector<std::pair<int, int64_t>> row;
    row.reserve(e - a);
    for (int t = a; t < e; ++t) row.push_back({c.csr_col[t], c.csr_src[t]});
    std::sort(row.begin(), row.end());
    for (int t = a; t < e; ++t) { c.csr_col[t] = row[t - a].first; c.csr_src[t] = row[t - a].second; }
  }
  // bricks of 64 points (4x4x4 blocks when the grid allows, else runs of
  // 64 consecutive points): the functions touching each brick, padded to a
  // multiple of 4 (the MFMA depth)
  BrickGeo& geo = c.geo;
  geo = BrickGeo{};
  {
    const int n1 = c.p.n[0], n2 = c.p.n[1], n3 = c.p.n[2];
    // 8 x 8 x 1 blocks: 64-byte runs of FP64 values per state row (4 x 4 x 4
    // cubes, denser still, leave 32-byte runs and were slower: the fused
    // scatter + projection 0.99 -> 1.28 ms on c2, 4.45 -> 6.5 ms on c3)
    (void)n3;
    if (n1 % 8 == 0 && n2 % 8 == 0) { geo.cube = 1; geo.lx = 3; geo.ly = 3; geo.lz = 0; }
    geo.n1 = n1;
    geo.n12 = (int64_t)n1 * n2;
    geo.nbx = n1 >> geo.lx;
    geo.nby = geo.cube ? n2 >> geo.ly : 1;
  }
  const int nbrick = geo.cube ? c.nd / kBrick : (c.nd + kBrick - 1) / kBrick;
  geo.nbrick = nbrick;
  auto brick_point = [&](int b, int i) -> int64_t { return geo.base(b) + geo.off(i); };   // >= nd: outside
  c.boff.assign(nbrick + 1, 0);
  c.bnj.assign(nbrick, 0);
  c.bj.clear();
  std::vector<int> js;
  for (int b = 0; b < nbrick; ++b) {
    js.clear();
    for (int i = 0; i < kBrick; ++i) {
      const int64_t p = brick_point(b, i);
      if (p >= c.nd) continue;
      for (int t = c.csr_ptr[p]; t < c.csr_ptr[p + 1]; ++t) js.push_back(c.csr_col[t]);
    }
    std::sort(js.begin(), js.end());
    js.erase(std::unique(js.begin(), js.end()), js.end());
    const int nj = (int)js.size();
    const int njp = (nj + 3) / 4 * 4;
    c.bnj[b] = nj;
    c.boff[b + 1] = c.boff[b] + njp;
    for (int t = 0; t < njp; ++t) c.bj.push_back(t < nj ? js[t] : -1);
  }
  // a tail past the last brick: a kernel may read a clamped index there
  c.bj.insert(c.bj.end(), 64, -1);
  c.bsrc.assign((size_t)c.boff[nbrick] * kBrick, -1);
  for (int b = 0; b < nbrick; ++b) {
    const int* bjb = c.bj.data() + c.boff[b];
    const int nj = c.bnj[b];
    for (int i = 0; i < kBrick; ++i) {
      const int64_t p = brick_point(b, i);
      if (p >= c.nd) continue;
      for (int t = c.csr_ptr[p]; t < c.csr_ptr[p + 1]; ++t) {
        const int jl = (int)(std::lower_bound(bjb, bjb + nj, c.csr_col[t]) - bjb);
        c.bsrc[(c.boff[b] + jl) * kBrick + i] = c.csr_src[t];
      }
    }
  }
  // projection bricks (bricks 4b .. 4b+3): the function list of each brick
  // is padded to a multiple of 16 (one matrix-core tile), and the value tile
  // is stored in operand order [tile][64-point piece][step group i][lane][G]:
  // at steps G i .. G i + G-1 lane l of a wave holds row 16 tile + l%16 at
  // the G local indices from 4G i + G (l/16) of the piece (consecutive in
  // memory), which is also the order in which the lane reads its state row.
  // G = 2 (16-byte groups in FP64 and complex FP32) unless every block is
  // real FP32 (G = 4).
  c.pgroup = (c.mixed && !c.any_complex) ? 4 : 2;
  const int G = c.pgroup;
  c.pboff.assign(1, 0);
  c.max_ptiles = 0;
  c.pbnj.clear();
  c.pbsrc.clear();
  c.pdest.clear();
  c.jrow.assign(c.nproj + 1, 0);
  {
    constexpr int P = kPBrick / kBrick;
    const int npb = (nbrick + P - 1) / P;
    std::vector<int> pbj;   // padded slots, -1 for padding
    for (int b = 0; b < npb; ++b) {
      js.clear();
      for (int piece = 0; piece < P && P * b + piece < nbrick; ++piece)
        for (int i = 0; i < kBrick; ++i) {
          const int64_t p = brick_point(P * b + piece, i);
          if (p >= c.nd) continue;
          for (int t = c.csr_ptr[p]; t < c.csr_ptr[p + 1]; ++t) js.push_back(c.csr_col[t]);
        }
      std::sort(js.begin(), js.end());
      js.erase(std::unique(js.begin(), js.end()), js.end());
      const int nj = (int)js.size();
      const int njp = (nj + 15) / 16 * 16;
      c.pbnj.push_back(nj);
      c.max_ptiles = std::max(c.max_ptiles, njp / 16);
      c.pboff.push_back(c.pboff.back() + njp);
      for (int t = 0; t < njp; ++t) {
        pbj.push_back(t < nj ? js[t] : -1);
        if (t < nj) ++c.jrow[js[t] + 1];
      }
    }
    for (int j = 0; j < c.nproj; ++j) c.jrow[j + 1] += c.jrow[j];
    c.pdest.assign(pbj.size(), -1);
    std::vector<int64_t> fill(c.jrow.begin(), c.jrow.end() - 1);
    for (size_t sl = 0; sl < pbj.size(); ++sl)
      if (pbj[sl] >= 0) c.pdest[sl] = fill[pbj[sl]]++;
    c.pbsrc.assign((size_t)c.pboff.back() * kPBrick, -1);
    for (int b = 0; b < npb; ++b) {
      const int* jb = pbj.data() + c.pboff[b];
      const int nj = c.pbnj[b];
      const int64_t tile0 = c.pboff[b] / 16;
      for (int piece = 0; piece < P && P * b + piece < nbrick; ++piece)
        for (int r = 0; r < kBrick; ++r) {
          const int64_t p = brick_point(P * b + piece, r);
          if (p >= c.nd) continue;
          const int i = r / (4 * G), q = (r % (4 * G)) / G, h = r % G;
          for (int t = c.csr_ptr[p]; t < c.csr_ptr[p + 1]; ++t) {
            const int jl = (int)(std::lower_bound(jb, jb + nj, c.csr_col[t]) - jb);
            const int64_t lane = q * 16 + jl % 16;
            const int64_t flat = ((((tile0 + jl / 16) * P + piece) * (16 / G) + i) * 64 + lane) * G + h;
            c.pbsrc[flat] = c.csr_src[t];
          }
        }
    }
  }
  return HCU_OK;
}

void fill_stencil_coef(const Ctx& c, int ik, StencilCoef& sc) {
  const int n0 = c.p.n0;
  sc.R = n0;
  double f = fact(n0) * fact(n0);
  sc.center = 0;
  for (int a = 0; a < 3; ++a) {
    sc.n[a] = c.p.n[a];
    double h2 = c.h[a] * c.h[a];
    double w0 = 0;
    for (int q = 1; q <= n0; ++q) w0 += 1.0 / (q * q);
    w0 *= -2.0 / h2;
    sc.kin[a][0] = -0.5 * w0;
    for (int q = 1; q <= kMaxR; ++q) {
      double w = 0;
      if (q <= n0) w = 2.0 * ((q % 2) ? 1.0 : -1.0) / (h2 * q * q) * f / (fact(n0 - q) * fact(n0 + q));
      sc.kin[a][q] = -0.5 * w;
    }
    sc.center += sc.kin[a][0];
    double kl = c.kpts[3 * ik + a] * c.p.L[a];
    sc.phase_re[a] = std::cos(kl);
    sc.phase_im[a] = std::sin(kl);
  }
}

// ------------------------------------------------------------------ device tables
struct AtomV { double x, y, z, depth, width; };

__global__ void k_vloc(double* V, float* Vf, const AtomV* atoms, int natom, int n1, int n2, int n3,
                       double h1, double h2, double h3, double L1, double L2, double L3) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t nd = (int64_t)n1 * n2 * n3;
  if (p >= nd) return;
  int i = (int)(p % n1), j = (int)((p / n1) % n2), k = (int)(p / ((int64_t)n1 * n2));
  double x = i * h1, y = j * h2, z = k * h3;
  double v = 0;
  for (int a = 0; a < natom; ++a) {
    AtomV at = atoms[a];
    double rcut2 = 2.0 * at.width * at.width * log(at.depth / 1e-17);
    double rcut = sqrt(rcut2);
    int m1 = (int)ceil(rcut / L1) + 1, m2 = (int)ceil(rcut / L2) + 1, m3 = (int)ceil(rcut / L3) + 1;
    double inv = 1.0 / (2 * at.width * at.width);
    for (int t3 = -m3; t3 <= m3; ++t3) {
      double dz = z - at.z - t3 * L3;
      if (dz * dz > rcut2) continue;
      for (int t2 = -m2; t2 <= m2; ++t2) {
        double dy = y - at.y - t2 * L2;
        if (dy * dy + dz * dz > rcut2) continue;
        for (int t1 = -m1; t1 <= m1; ++t1) {
          double dx = x - at.x - t1 * L1;
          double r2 = dx * dx + dy * dy + dz * dz;
          if (r2 <= rcut2) v -= at.depth * exp(-r2 * inv);
        }
      }
    }
  }
  V[p] = v;
  if (Vf) Vf[p] = (float)v;
}

// Values of one block's functions on its support, summed over periodic images
// with Bloch phase e^{+i k.T} (T = image translation).  moment = 0, 1, 2:
// the moment functions of the Hubbard blocks instead, every image term times
// its own displacement component (x - R - T)_moment (KB blocks get zeros).
template <typename T>
__global__ void k_block_values(const BlockDesc* blocks, const int* supp, T* val, int n1, int n2,
                               double h1, double h2, double h3, double L1, double L2, double L3,
                               double k1, double k2, double k3, int moment) {
  const BlockDesc b = blocks[blockIdx.y];
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= b.nsupp) return;
  if (moment >= 0 && b.type == 0) {
    for (int m = 0; m < b.nm; ++m) val[b.val_off + (int64_t)m * b.nsupp + q] = T(0);
    return;
  }
  int pt = supp[b.supp_off + q];
  int i = pt % n1, j = (pt / n1) % n2, k = pt / (n1 * n2);
  double x = i * h1, y = j * h2, z = k * h3;
  double rmax = 0;
  for (int ch = 0; ch < b.nchan; ++ch) rmax = fmax(rmax, b.chan_rc[ch]);
  int m1 = (int)ceil(rmax / L1) + 1, m2 = (int)ceil(rmax / L2) + 1, m3 = (int)ceil(rmax / L3) + 1;
  double acc_re[kMaxNm], acc_im[kMaxNm];
  for (int m = 0; m < kMaxNm; ++m) { acc_re[m] = 0; acc_im[m] = 0; }
  double ylm[5];
  for (int t3 = -m3; t3 <= m3; ++t3)
    for (int t2 = -m2; t2 <= m2; ++t2)
      for (int t1 = -m1; t1 <= m1; ++t1) {
        double dx = x - b.center[0] - t1 * L1, dy = y - b.center[1] - t2 * L2, dz = z - b.center[2] - t3 * L3;
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r > rmax) continue;
        double ph = k1 * t1 * L1 + k2 * t2 * L2 + k3 * t3 * L3;
        double cr = cos(ph), ci = sin(ph);
        int m0 = 0;
        for (int ch = 0; ch < b.nchan; ++ch) {
          int l = b.chan_l[ch];
          if (r <= b.chan_rc[ch]) {
            double rad = (b.type == 0) ? kb_radial(r, b.chan_norm[ch], l, b.width)
                                       : hub_radial(r, b.chan_norm[ch], b.power, b.alpha);
            real_ylm(l, dx, dy, dz, ylm);
            const double w = moment == 0 ? dx : moment == 1 ? dy : moment == 2 ? dz : 1.0;
            for (int m = 0; m < 2 * l + 1; ++m) {
              acc_re[m0 + m] += rad * ylm[m] * w * cr;
              acc_im[m0 + m] += rad * ylm[m] * w * ci;
            }
          }
          m0 += 2 * l + 1;
        }
      }
  for (int m = 0; m < b.nm; ++m) val[b.val_off + (int64_t)m * b.nsupp + q] = make_scalar<T>(acc_re[m], acc_im[m]);
}

// Cyclic Jacobi eigen-decomposition of a small real symmetric matrix (n <= 10),
// then A^{-1/2} = V diag(lam^{-1/2}) V^T written over A.
__device__ void jacobi_inv_sqrt(double* A, int n) {
  double V[100];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i * n + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
    if (off < 1e-34) break;
    for (int pq = 0; pq < n * n; ++pq) {
      int pp = pq / n, qq = pq % n;
      if (qq <= pp) continue;
      double apq = A[pp * n + qq];
      if (fabs(apq) < 1e-300) continue;
      double theta = (A[qq * n + qq] - A[pp * n + pp]) / (2 * apq);
      double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1));
      double cs = 1 / sqrt(t * t + 1), sn = t * cs;
      for (int r = 0; r < n; ++r) {   // columns p, q
        double arp = A[r * n + pp], arq = A[r * n + qq];
        A[r * n + pp] = cs * arp - sn * arq;
        A[r * n + qq] = sn * arp + cs * arq;
      }
      for (int r = 0; r < n; ++r) {   // rows p, q
        double apr = A[pp * n + r], aqr = A[qq * n + r];
        A[pp * n + r] = cs * apr - sn * aqr;
        A[qq * n + r] = sn * apr + cs * aqr;
      }
      for (int r = 0; r < n; ++r) {
        double vrp = V[r * n + pp], vrq = V[r * n + qq];
        V[r * n + pp] = cs * vrp - sn * vrq;
        V[r * n + qq] = sn * vrp + cs * vrq;
      }
    }
  }
  double lam[10];
  for (int i = 0; i < n; ++i) lam[i] = 1.0 / sqrt(A[i * n + i]);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0;
      for (int k = 0; k < n; ++k) s += V[i * n + k] * lam[k] * V[j * n + k];
      A[i * n + j] = s;
    }
}

// Loewdin step for the Hubbard blocks: O = Phi^H Phi dV, Phi <- Phi O^{-1/2}.
// One workgroup per Hubbard block.  Complex O is handled through its real
// symmetric embedding [[Re, -Im], [Im, Re]], whose inverse square root embeds
// the complex one.
template <typename T>
__global__ void k_lowdin(const BlockDesc* blocks, const int* hub_blocks, T* val, double dv, double* Cout) {
  using R = typename real_of<T>::type;
  const BlockDesc b = blocks[hub_blocks[blockIdx.x]];
  const int nm = b.nm;
  __shared__ double sO_re[25], sO_im[25];
  __shared__ double red[256];
  __shared__ double M[100];
  T* v = val + b.val_off;
  for (int e = 0; e < nm * nm; ++e) {
    int m = e / nm, mp = e % nm;
    double sr = 0, si = 0;
    for (int q = threadIdx.x; q < b.nsupp; q += blockDim.x) {
      T a = v[(int64_t)m * b.nsupp + q], bb = v[(int64_t)mp * b.nsupp + q];
      T prod = mul_conj(bb, a);   // conj(phi_m) phi_m'
      if constexpr (sizeof(T) == sizeof(R)) { sr += (double)prod; }
      else { sr += (double)prod.re; si += (double)prod.im; }
    }
    red[threadIdx.x] = sr;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) { if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s]; __syncthreads(); }
    if (threadIdx.x == 0) sO_re[e] = red[0] * dv;
    __syncthreads();
    red[threadIdx.x] = si;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) { if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s]; __syncthreads(); }
    if (threadIdx.x == 0) sO_im[e] = red[0] * dv;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const bool cp = sizeof(T) != sizeof(R);
    int n = cp ? 2 * nm : nm;
    for (int i = 0; i < nm; ++i)
      for (int j = 0; j < nm; ++j) {
        // Hermitise
        double re = 0.5 * (sO_re[i * nm + j] + sO_re[j * nm + i]);
        double im = 0.5 * (sO_im[i * nm + j] - sO_im[j * nm + i]);
        if (!cp) { M[i * n + j] = re; continue; }
        M[i * n + j] = re;            M[i * n + (j + nm)] = -im;
        M[(i + nm) * n + j] = im;     M[(i + nm) * n + (j + nm)] = re;
      }
    jacobi_inv_sqrt(M, n);
    for (int i = 0; i < nm; ++i)
      for (int j = 0; j < nm; ++j) {
        sO_re[i * nm + j] = M[i * n + j];
        sO_im[i * nm + j] = cp ? M[(i + nm) * n + j] : 0.0;
      }
    if (Cout)   // the coefficients, kept for the moment functions
      for (int e = 0; e < nm * nm; ++e) {
        Cout[50 * blockIdx.x + e] = sO_re[e];
        Cout[50 * blockIdx.x + 25 + e] = sO_im[e];
      }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < b.nsupp; q += blockDim.x) {
    T old[5];
    for (int m = 0; m < nm; ++m) old[m] = v[(int64_t)m * b.nsupp + q];
    for (int m = 0; m < nm; ++m) {
      T s = T(0);
      for (int mp = 0; mp < nm; ++mp)
        s += make_scalar<T>(sO_re[mp * nm + m], sO_im[mp * nm + m]) * old[mp];
      v[(int64_t)m * b.nsupp + q] = s;
    }
  }
}

// The stored Loewdin coefficients C of each Hubbard block (re at [0, 25),
// im at [25, 50) of the block's record) applied to other values on the same
// support: v_m <- sum_m' C_m'm v_m' (as k_lowdin applies them to the orbitals).
template <typename T>
__global__ void k_apply_lowdin(const BlockDesc* blocks, const int* hub_blocks, T* val, const double* C) {
  const BlockDesc b = blocks[hub_blocks[blockIdx.x]];
  const int nm = b.nm;
  const double* cr = C + 50 * blockIdx.x;
  const double* ci = cr + 25;
  T* v = val + b.val_off;
  for (int q = threadIdx.x; q < b.nsupp; q += blockDim.x) {
    T old[5];
    for (int m = 0; m < nm; ++m) old[m] = v[(int64_t)m * b.nsupp + q];
    for (int m = 0; m < nm; ++m) {
      T acc = T(0);
      for (int mp = 0; mp < nm; ++mp) acc += make_scalar<T>(cr[mp * nm + m], ci[mp * nm + m]) * old[mp];
      v[(int64_t)m * b.nsupp + q] = acc;
    }
  }
}

template <typename T>
__global__ void k_gather_csr(const T* csc, const int64_t* src, T* csr, int64_t nnz) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) csr[e] = src[e] >= 0 ? csc[src[e]] : T(0);
}

template <typename T>
static hcu_status tables_for(Ctx& c) {
  hipStream_t st = c.stream;
  int nblk = (int)c.blocks.size();
  int maxs = 0;
  for (auto& b : c.blocks) maxs = std::max(maxs, b.nsupp);
  std::vector<int> hub_blocks;
  for (int i = 0; i < nblk; ++i) if (c.blocks[i].type == 1) hub_blocks.push_back(i);
  int* d_hb = (int*)c.d_red;   // scratch (sized >= nblocks ints)
  if (!hub_blocks.empty())
    HCU_HIP(hipMemcpyAsync(d_hb, hub_blocks.data(), hub_blocks.size() * sizeof(int), hipMemcpyHostToDevice, st));
  for (int ik = 0; ik < c.p.nk; ++ik) {
    T* cscv = (T*)c.d_cscv[ik];
    if (nblk > 0 && maxs > 0) {
      dim3 grid((maxs + 127) / 128, nblk);
      k_block_values<T><<<grid, 128, 0, st>>>(c.d_blocks, c.d_supp, cscv, c.p.n[0], c.p.n[1], c.h[0], c.h[1],
                                              c.h[2], c.p.L[0], c.p.L[1], c.p.L[2], c.kpts[3 * ik],
                                              c.kpts[3 * ik + 1], c.kpts[3 * ik + 2], -1);
      HCU_HIP(hipGetLastError());
    }
    if (c.p.lowdin && !hub_blocks.empty()) {
      k_lowdin<T><<<(int)hub_blocks.size(), 256, 0, st>>>(c.d_blocks, d_hb, cscv, c.dv,
                                                          c.d_lowC + (size_t)ik * hub_blocks.size() * 50);
      HCU_HIP(hipGetLastError());
    }
    const int64_t nbv = (int64_t)c.bsrc.size();
    if (nbv > 0) {
      k_gather_csr<T><<<(unsigned)((nbv + 255) / 256), 256, 0, st>>>(cscv, c.d_bsrc, (T*)c.d_bval[ik], nbv);
      HCU_HIP(hipGetLastError());
    }
    const int64_t npv = (int64_t)c.pbsrc.size();
    if (npv > 0) {
      k_gather_csr<T><<<(unsigned)((npv + 255) / 256), 256, 0, st>>>(cscv, c.d_pbsrc, (T*)c.d_pbval[ik], npv);
      HCU_HIP(hipGetLastError());
    }
  }
  HCU_HIP(hipStreamSynchronize(st));   // hub_blocks (host) must outlive its copy
  return HCU_OK;
}

// Moment functions of the Hubbard orbitals at k-point ik, direction b, in
// the projection-brick layout: values on each block's support (KB blocks
// zero) into `csc` (nval elements), the orbitals' Loewdin coefficients
// applied, then gathered into `table` (the layout of d_pbval).
template <typename T>
hcu_status build_moment_table(Ctx& c, int ik, int b, T* csc, T* table, hipStream_t st) {
  const int nblk = (int)c.blocks.size();
  const int nh = (int)c.hub_atoms.size();
  int maxs = 0;
  for (auto& bl : c.blocks) maxs = std::max(maxs, bl.nsupp);
  if (nblk == 0 || maxs == 0 || nh == 0) return HCU_OK;
  dim3 grid((maxs + 127) / 128, nblk);
  k_block_values<T><<<grid, 128, 0, st>>>(c.d_blocks, c.d_supp, csc, c.p.n[0], c.p.n[1], c.h[0], c.h[1], c.h[2],
                                          c.p.L[0], c.p.L[1], c.p.L[2], c.kpts[3 * ik], c.kpts[3 * ik + 1],
                                          c.kpts[3 * ik + 2], b);
  HCU_HIP(hipGetLastError());
  if (c.p.lowdin) {
    k_apply_lowdin<T><<<nh, 256, 0, st>>>(c.d_blocks, c.d_hub_blocks, csc, c.d_lowC + (size_t)ik * nh * 50);
    HCU_HIP(hipGetLastError());
  }
  const int64_t npv = (int64_t)c.pbsrc.size();
  if (npv > 0) {
    k_gather_csr<T><<<(unsigned)((npv + 255) / 256), 256, 0, st>>>(csc, c.d_pbsrc, table, npv);
    HCU_HIP(hipGetLastError());
  }
  return HCU_OK;
}
template hcu_status build_moment_table<double>(Ctx&, int, int, double*, double*, hipStream_t);
template hcu_status build_moment_table<float>(Ctx&, int, int, float*, float*, hipStream_t);
template hcu_status build_moment_table<cplx<double>>(Ctx&, int, int, cplx<double>*, cplx<double>*, hipStream_t);
template hcu_status build_moment_table<cplx<float>>(Ctx&, int, int, cplx<float>*, cplx<float>*, hipStream_t);

hcu_status device_tables(Ctx& c) {
  hipStream_t st = c.stream;
  // local potential
  std::vector<AtomV> av(c.p.natom);
  for (int a = 0; a < c.p.natom; ++a) {
    const hcu_species& s = c.species[c.atom_species[a]];
    av[a] = {c.pos[3 * a], c.pos[3 * a + 1], c.pos[3 * a + 2], s.vloc_depth, s.vloc_width};
  }
  AtomV* d_av = (AtomV*)c.d_red;
  HCU_HIP(hipMemcpyAsync(d_av, av.data(), av.size() * sizeof(AtomV), hipMemcpyHostToDevice, st));
  // with the density-dependent Hamiltonian V_loc is kept apart; the total
  // potential is assembled from it afterwards
  k_vloc<<<(c.nd + 255) / 256, 256, 0, st>>>(c.hxc ? c.d_Vloc : c.d_V, (c.mixed && !c.hxc) ? c.d_Vf : nullptr, d_av,
                                             c.p.natom, c.p.n[0],
                                             c.p.n[1], c.p.n[2], c.h[0], c.h[1], c.h[2], c.p.L[0], c.p.L[1],
                                             c.p.L[2]);
  HCU_HIP(hipGetLastError());
  HCU_HIP(hipStreamSynchronize(st));   // d_red is reused below
  if (!c.supp.empty())
    HCU_HIP(hipMemcpyAsync(c.d_supp, c.supp.data(), c.supp.size() * sizeof(int), hipMemcpyHostToDevice, st));
  if (!c.blocks.empty())
    HCU_HIP(hipMemcpyAsync(c.d_blocks, c.blocks.data(), c.blocks.size() * sizeof(BlockDesc), hipMemcpyHostToDevice, st));
  auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
  };
  HCU_HIP(up(c.d_boff, c.boff.data(), c.boff.size() * sizeof(int64_t)));
  HCU_HIP(up(c.d_bnj, c.bnj.data(), c.bnj.size() * sizeof(int)));
  HCU_HIP(up(c.d_bj, c.bj.data(), c.bj.size() * sizeof(int)));
  HCU_HIP(up(c.d_bsrc, c.bsrc.data(), c.bsrc.size() * sizeof(int64_t)));
  HCU_HIP(up(c.d_pboff, c.pboff.data(), c.pboff.size() * sizeof(int64_t)));
  HCU_HIP(up(c.d_pbnj, c.pbnj.data(), c.pbnj.size() * sizeof(int)));
  HCU_HIP(up(c.d_pbsrc, c.pbsrc.data(), c.pbsrc.size() * sizeof(int64_t)));
  HCU_HIP(up(c.d_pdest, c.pdest.data(), c.pdest.size() * sizeof(int64_t)));
  HCU_HIP(up(c.d_jrow, c.jrow.data(), c.jrow.size() * sizeof(int64_t)));
  hcu_status s;
  if (c.any_complex) s = c.mixed ? tables_for<cplx<float>>(c) : tables_for<cplx<double>>(c);
  else s = c.mixed ? tables_for<float>(c) : tables_for<double>(c);
  if (s != HCU_OK) return s;
  HCU_HIP(hipStreamSynchronize(st));
  return HCU_OK;
}

}  // namespace hcu
