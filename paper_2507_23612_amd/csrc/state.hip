// Snapshot and restore of a context's SCF state (resume after an
// interruption): input occupation matrices and the mixing history, the
// iteration counter and convergence bookkeeping, the filter bounds of every
// (spin, k) block, the last eigenvalues/occupations/energies and the
// orbital blocks themselves; with the density-dependent Hamiltonian also
// the input density and the density mixing window, and the rotated
// projections of the blocks (the next filter starts from them).  A restored
// context continues the SCF exactly
// as the saved one would have (the next step filters the restored blocks
// with the restored bounds and mixes with the restored history).
#include "common.h"

#include <cstring>

using namespace hcu;

namespace {
constexpr char kMagic[8] = {'H', 'C', 'U', 'S', 'T', 'A', 'T', 'E'};
constexpr uint32_t kVersion = 3;

struct StateHeader {
  char magic[8];
  uint32_t version;
  int32_t nd, ns, nspin, nk, nhub, mixed, complex_, elem;
  int32_t scf_iter, scf_ready, have_old, have_results;
  int32_t n_hist, vec_len;
  int32_t hxc, n_rho_hist;
  double F_old;
  hcu_scf_opts opts;
  hcu_energies en;
};

// rotated projections: one validity flag (a double) and the [ns][nproj]
// block per (spin, k)
size_t px_bytes(const Ctx& c) {
  const int nsk = c.p.nspin * c.p.nk;
  const size_t es = (c.mixed ? 4 : 8) * (c.any_complex ? 2 : 1);
  return (size_t)nsk * (sizeof(double) + es * (size_t)c.p.ns * c.nproj);
}

size_t state_bytes(const Ctx& c, size_t* hist_len) {
  const int nsk = c.p.nspin * c.p.nk;
  const size_t nh = c.mix_x.size();
  const size_t vl = nh ? c.mix_x[0].size() : 0;
  if (hist_len) *hist_len = vl;
  const size_t es = (c.mixed ? 4 : 8) * (c.any_complex ? 2 : 1);
  const size_t hx = c.hxc ? (size_t)c.nd * (2 + 2 * c.hxc_slots.size()) + (c.mixed ? (c.nd + 1) / 2 : 0) : 0;
  return sizeof(StateHeader) + sizeof(double) * (2 * c.D_in.size() + c.bounds.size() + 2 * (size_t)nsk * c.p.ns +
                                                 2 * nh * vl + hx) +
         (size_t)nsk * es * c.nd * c.p.ns + px_bytes(c);
}

template <typename V>
void put(char*& p, const V* v, size_t n) {
  std::memcpy(p, v, sizeof(V) * n);
  p += sizeof(V) * n;
}
template <typename V>
void get(const char*& p, V* v, size_t n) {
  std::memcpy(v, p, sizeof(V) * n);
  p += sizeof(V) * n;
}
}  // namespace

extern "C" {

hcu_status hcu_state_size(const hcu_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return HCU_INVALID_ARG;
  if (!ctx->bound) return HCU_NOT_BOUND;
  *bytes = state_bytes(*ctx, nullptr);
  return HCU_OK;
}

hcu_status hcu_save_state(hcu_ctx* ctx, void* host, size_t bytes) {
  if (!ctx || !host) return HCU_INVALID_ARG;
  Ctx& c = *ctx;
  if (!c.bound) return HCU_NOT_BOUND;
  size_t vl = 0;
  if (bytes < state_bytes(c, &vl)) {
    c.err = "state buffer too small (see hcu_state_size)";
    return HCU_INVALID_ARG;
  }
  const int nsk = c.p.nspin * c.p.nk;
  StateHeader h{};
  std::memcpy(h.magic, kMagic, 8);
  h.version = kVersion;
  h.nd = c.nd;
  h.ns = c.p.ns;
  h.nspin = c.p.nspin;
  h.nk = c.p.nk;
  h.nhub = (int)c.hub_atoms.size();
  h.mixed = c.mixed ? 1 : 0;
  h.complex_ = c.any_complex ? 1 : 0;
  h.elem = (int)((c.mixed ? 4 : 8) * (c.any_complex ? 2 : 1));
  h.scf_iter = c.scf_iter;
  h.scf_ready = c.scf_ready ? 1 : 0;
  h.have_old = c.scf_have_old ? 1 : 0;
  h.have_results = c.have_results ? 1 : 0;
  h.n_hist = (int)c.mix_x.size();
  h.vec_len = (int)vl;
  h.hxc = c.hxc ? 1 : 0;
  h.n_rho_hist = c.hxc ? (int)c.hxc_slots.size() : 0;
  h.F_old = c.scf_F_old;
  h.opts = c.scf_opts;
  h.en = c.en;
  char* p = static_cast<char*>(host);
  put(p, &h, 1);
  std::vector<double> lam(c.lam), occ(c.occ);
  lam.resize((size_t)nsk * c.p.ns, 0.0);
  occ.resize((size_t)nsk * c.p.ns, 0.0);
  std::vector<double> dout(c.D_out);
  dout.resize(c.D_in.size(), 0.0);
  put(p, c.D_in.data(), c.D_in.size());
  put(p, dout.data(), dout.size());
  put(p, c.bounds.data(), c.bounds.size());
  put(p, lam.data(), lam.size());
  put(p, occ.data(), occ.size());
  for (size_t i = 0; i < c.mix_x.size(); ++i) put(p, c.mix_x[i].data(), vl);
  for (size_t i = 0; i < c.mix_f.size(); ++i) put(p, c.mix_f[i].data(), vl);
  const size_t blk = (size_t)h.elem * c.nd * c.p.ns;
  for (int sk = 0; sk < nsk; ++sk) {
    HCU_HIP(hipMemcpyAsync(p, c.d_X[sk], blk, hipMemcpyDeviceToHost, c.stream));
    p += blk;
  }
  const size_t pblk = (size_t)h.elem * c.p.ns * c.nproj;
  for (int sk = 0; sk < nsk; ++sk) {
    const double f = (sk < (int)c.px_valid.size() && c.px_valid[sk]) ? 1.0 : 0.0;
    put(p, &f, 1);
    if (pblk) HCU_HIP(hipMemcpyAsync(p, c.d_PX[sk], pblk, hipMemcpyDeviceToHost, c.stream));
    p += pblk;
  }
  if (c.hxc) {
    // the potential as it stands (recomputing it from rho_in would round differently)
    const size_t vb = sizeof(double) * c.nd;
    HCU_HIP(hipMemcpyAsync(p, c.d_V, vb, hipMemcpyDeviceToHost, c.stream));
    p += vb;
    if (c.mixed) {
      HCU_HIP(hipMemcpyAsync(p, c.d_Vf, sizeof(float) * c.nd, hipMemcpyDeviceToHost, c.stream));
      p += sizeof(double) * ((c.nd + 1) / 2);
    }
    HCU_HIP(hipMemcpyAsync(p, c.d_rho_in, vb, hipMemcpyDeviceToHost, c.stream));
    p += vb;
    for (int slot : c.hxc_slots) {
      HCU_HIP(hipMemcpyAsync(p, c.d_hx + (size_t)slot * c.nd, vb, hipMemcpyDeviceToHost, c.stream));
      p += vb;
      HCU_HIP(hipMemcpyAsync(p, c.d_hf + (size_t)slot * c.nd, vb, hipMemcpyDeviceToHost, c.stream));
      p += vb;
    }
  }
  HCU_HIP(hipStreamSynchronize(c.stream));
  return HCU_OK;
}

hcu_status hcu_load_state(hcu_ctx* ctx, const void* host, size_t bytes) {
  if (!ctx || !host) return HCU_INVALID_ARG;
  Ctx& c = *ctx;
  if (!c.bound) return HCU_NOT_BOUND;
  if (bytes < sizeof(StateHeader)) {
    c.err = "state buffer too small";
    return HCU_INVALID_ARG;
  }
  const char* p = static_cast<const char*>(host);
  StateHeader h;
  get(p, &h, 1);
  const int nsk = c.p.nspin * c.p.nk;
  if (std::memcmp(h.magic, kMagic, 8) != 0 || h.version != kVersion) {
    c.err = "not a saved state of this library version";
    return HCU_INVALID_ARG;
  }
  if (h.nd != c.nd || h.ns != c.p.ns || h.nspin != c.p.nspin || h.nk != c.p.nk ||
      h.nhub != (int)c.hub_atoms.size() || h.mixed != (c.mixed ? 1 : 0) || h.complex_ != (c.any_complex ? 1 : 0)) {
    c.err = "saved state belongs to a problem of another shape or precision";
    return HCU_INVALID_ARG;
  }
  if (h.hxc != (c.hxc ? 1 : 0)) {
    c.err = "saved state belongs to a problem with another Hamiltonian (hxc flag)";
    return HCU_INVALID_ARG;
  }
  if (h.n_hist < 0 || h.vec_len < 0 || h.n_hist > 1024 || h.n_rho_hist < 0 || h.n_rho_hist > kHxcWindow ||
      (!c.hxc && h.n_rho_hist != 0)) {
    c.err = "corrupt saved state";
    return HCU_INVALID_ARG;
  }
  const size_t need = sizeof(StateHeader) +
                      sizeof(double) * (2 * c.D_in.size() + c.bounds.size() + 2 * (size_t)nsk * c.p.ns +
                                        2 * (size_t)h.n_hist * h.vec_len +
                                        (c.hxc ? (size_t)c.nd * (2 + 2 * (size_t)h.n_rho_hist) +
                                                     (c.mixed ? (c.nd + 1) / 2 : 0)
                                               : 0)) +
                      (size_t)nsk * h.elem * c.nd * c.p.ns + px_bytes(c);
  if (bytes < need) {
    c.err = "saved state truncated";
    return HCU_INVALID_ARG;
  }
  std::vector<double> din(c.D_in.size());
  get(p, din.data(), din.size());
  c.D_out.assign(c.D_in.size(), 0.0);
  get(p, c.D_out.data(), c.D_out.size());
  get(p, c.bounds.data(), c.bounds.size());
  c.lam.assign((size_t)nsk * c.p.ns, 0.0);
  c.occ.assign((size_t)nsk * c.p.ns, 0.0);
  get(p, c.lam.data(), c.lam.size());
  get(p, c.occ.data(), c.occ.size());
  c.mix_x.assign(h.n_hist, std::vector<double>(h.vec_len));
  c.mix_f.assign(h.n_hist, std::vector<double>(h.vec_len));
  for (auto& v : c.mix_x) get(p, v.data(), v.size());
  for (auto& v : c.mix_f) get(p, v.data(), v.size());
  const size_t blk = (size_t)h.elem * c.nd * c.p.ns;
  for (int sk = 0; sk < nsk; ++sk) {
    HCU_HIP(hipMemcpyAsync(c.d_X[sk], p, blk, hipMemcpyHostToDevice, c.stream));
    p += blk;
  }
  const size_t pblk = (size_t)h.elem * c.p.ns * c.nproj;
  c.px_valid.assign(nsk, 0);
  for (int sk = 0; sk < nsk; ++sk) {
    double f = 0.0;
    get(p, &f, 1);
    c.px_valid[sk] = (f != 0.0 && pblk) ? 1 : 0;
    if (pblk) HCU_HIP(hipMemcpyAsync(c.d_PX[sk], p, pblk, hipMemcpyHostToDevice, c.stream));
    p += pblk;
  }
  if (c.hxc) {
    const size_t vb = sizeof(double) * c.nd;
    HCU_HIP(hipMemcpyAsync(c.d_V, p, vb, hipMemcpyHostToDevice, c.stream));
    p += vb;
    if (c.mixed) {
      HCU_HIP(hipMemcpyAsync(c.d_Vf, p, sizeof(float) * c.nd, hipMemcpyHostToDevice, c.stream));
      p += sizeof(double) * ((c.nd + 1) / 2);
    }
    HCU_HIP(hipMemcpyAsync(c.d_rho_in, p, vb, hipMemcpyHostToDevice, c.stream));
    p += vb;
    c.hxc_slots.clear();
    for (int i = 0; i < h.n_rho_hist; ++i) {
      HCU_HIP(hipMemcpyAsync(c.d_hx + (size_t)i * c.nd, p, vb, hipMemcpyHostToDevice, c.stream));
      p += vb;
      HCU_HIP(hipMemcpyAsync(c.d_hf + (size_t)i * c.nd, p, vb, hipMemcpyHostToDevice, c.stream));
      p += vb;
      c.hxc_slots.push_back(i);
    }
    c.hxc_have_rho = true;
  }
  HCU_HIP(hipMemcpyAsync(c.d_lam, c.lam.data(), sizeof(double) * c.lam.size(), hipMemcpyHostToDevice, c.stream));
  HCU_HIP(hipMemcpyAsync(c.d_occ, c.occ.data(), sizeof(double) * c.occ.size(), hipMemcpyHostToDevice, c.stream));
  HCU_HIP(hipStreamSynchronize(c.stream));
  c.scf_iter = h.scf_iter;
  c.scf_ready = h.scf_ready != 0;
  c.scf_have_old = h.have_old != 0;
  c.have_results = h.have_results != 0;
  c.scf_F_old = h.F_old;
  c.scf_opts = h.opts;
  c.en = h.en;
  return hcu_set_hubbard_occupation(ctx, din.data());
}

}  // extern "C"
