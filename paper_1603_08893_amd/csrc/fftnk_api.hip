// Host driver and C-ABI of libfftnk (declared in include/fftnk.h).
//
// The driver runs Algorithm 1 of de Geus et al. (2017) for one load increment:
// boundary-condition solve with the tangent of the start state (Sec. 3.1),
// Newton iterations on G:K:dF = -G:P (Sec. 2.6) each solved by CG, the
// convergence test ||dF|| / ||F_t + dFbar|| < eta_NW after at least two solves,
// and the transactional commit of the converged state ("store converged
// state", Alg. 1).  All field work runs in the kernels of fftnk_kernels.hip; the
// host only sequences launches and reads back a few scalars per Newton
// iteration and per batch of CG iterations.
#include "fftnk.h"
#include "fftnk_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

using namespace fftnk;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Radix plan: powers of two in as few stages of 8 / 4 / 2 as possible, then
// 3, 5, 7 and any remaining prime (direct-sum stage).
bool make_plan(int n, AxisPlan& pl) {
  pl.n = n;
  pl.nstages = 0;
  int m = n, e2 = 0;
  while (m % 2 == 0) {
    m /= 2;
    ++e2;
  }
  if (e2 > 0) {
    const int ns = (e2 + 2) / 3;
    // distribute e2 bits over ns stages as evenly as possible (each <= 3)
    std::vector<int> b(ns, e2 / ns);
    for (int s = 0; s < e2 % ns; ++s) b[s] += 1;
    for (int s = 0; s < ns; ++s) {
      if (pl.nstages >= kMaxStages) return false;
      pl.radix[pl.nstages++] = 1 << b[s];
    }
  }
  for (int p = 3; m > 1; p += 2) {
    while (m % p == 0) {
      if (pl.nstages >= kMaxStages) return false;
      pl.radix[pl.nstages++] = p;
      m /= p;
    }
  }
  return true;
}

int largest_pow2_leq(int x) {
  int p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}

// pencils per work-group in the a1 / a0 passes: contiguous rows of at least
// 128 bytes where possible, within the LDS (60 KiB) and register (8 points per
// thread in pass 3) budgets.
int pick_m(int h, int nmax, size_t csz, int pref) {
  int m = std::min(pref, largest_pow2_leq(std::max(1, h)));
  while (m > 1 && ((size_t)nmax * m > (size_t)8 * kThreads || csz * ((size_t)nmax + 2 * (size_t)nmax * m) > 61440))
    m /= 2;
  return m;
}

}  // namespace

struct fftnk_ctx {
  int nrve = 0;
  int prec = PREC_F64;
  hipStream_t stream = nullptr;
  std::vector<Grid> g;
  long long ntot = 0;   // voxels over all RVEs
  long long nspec = 0;  // complex spectrum entries over all RVEs (9 components included)
  long long pstride = 0;
  std::vector<int> tw_len, tw_off;
  int tw_total = 0;
  // workspace layout (byte offsets)
  size_t o_Ft, o_F, o_P, o_x, o_r, o_p, o_w, o_F32, o_spec, o_phase, o_mu, o_mtab, o_part, o_cg, o_red, o_tw64,
      o_tw32, total = 0;
  char* ws = nullptr;
  bool have_phase = false, have_mat = false, use_mu = false;
  int model = MODEL_SVK, nphase = 0;
  double mtab[kMaxPhase * 4] = {};
  double* pinned = nullptr;  // host staging for device -> host scalars
  std::vector<double> Fbar_t;  // committed macroscopic F per RVE (host copy, informative)

  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
  size_t vsz() const { return prec == PREC_F64 ? sizeof(double) : sizeof(float); }
  double* Ft() const { return at<double>(o_Ft); }
  double* F() const { return at<double>(o_F); }
  double* P() const { return at<double>(o_P); }
  void* x() const { return ws + o_x; }
  void* r() const { return ws + o_r; }
  void* p() const { return ws + o_p; }
  void* w() const { return ws + o_w; }
  float* F32() const { return prec == PREC_F32 ? at<float>(o_F32) : nullptr; }
  void* spec() const { return ws + o_spec; }
  CgState* cg(int r) const { return at<CgState>(o_cg) + r; }
  double* red() const { return at<double>(o_red); }

  PassArgs args(int r) const {
    PassArgs a;
    a.g = g[r];
    a.tw64 = ws + o_tw64;
    a.tw32 = ws + o_tw32;
    a.partials = at<double>(o_part);
    a.pstride = pstride;
    a.slot_base = 0;
    return a;
  }
  Material material() const {
    Material m;
    m.phase = at<uint8_t>(o_phase);
    m.mu_field = use_mu ? at<double>(o_mu) : nullptr;
    m.table = at<double>(o_mtab);
    m.model = model;
    m.nphase = nphase;
    return m;
  }
};

namespace {

#define HIP_TRY(expr)                          \
  do {                                         \
    if ((expr) != hipSuccess) return FFTNK_EHIP; \
  } while (0)

int check_launch() { return hipGetLastError() == hipSuccess ? FFTNK_OK : FFTNK_EHIP; }

int fetch(fftnk_ctx* c, const void* dev, size_t bytes) {
  HIP_TRY(hipMemcpyAsync(c->pinned, dev, bytes, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return FFTNK_OK;
}

int init_ctx(fftnk_ctx* c, int nrve, const int* dims, int precision, void* stream) {
  if (nrve < 1 || nrve > kMaxRve || !dims) return FFTNK_EINVAL;
  if (precision != FFTNK_FP64 && precision != FFTNK_FP32_MIXED) return FFTNK_EINVAL;
  c->nrve = nrve;
  c->prec = precision == FFTNK_FP64 ? PREC_F64 : PREC_F32;
  c->stream = static_cast<hipStream_t>(stream);
  long long vox = 0, spec = 0, pmax = kRedBlocks;
  for (int r = 0; r < nrve; ++r) {
    Grid g{};
    g.n0 = dims[3 * r];
    g.n1 = dims[3 * r + 1];
    g.n2 = dims[3 * r + 2];
    for (int d = 0; d < 3; ++d) {
      const int nd = dims[3 * r + d];
      if (nd < 2 || nd > kMaxLen) return nd > kMaxLen ? FFTNK_EUNSUPPORTED : FFTNK_EINVAL;
      if (!make_plan(nd, g.ax[d])) return FFTNK_EUNSUPPORTED;
    }
    g.h = (g.n2 % 2 == 0) ? g.n2 / 2 : (g.n2 + 1) / 2;
    g.n = (long long)g.n0 * g.n1 * g.n2;
    g.rows = (long long)g.n0 * g.n1;
    g.vox_off = vox;
    g.spec_off = spec;
    g.inv_n = 1.0 / (double)g.n;
    g.rt = std::max(1, kThreads / g.n2);
    const int nmax = std::max(g.n0, g.n1);
    g.m64 = pick_m(g.h, nmax, 16, 8);
    g.m32 = pick_m(g.h, nmax, 8, 16);
    vox += g.n;
    spec += 9LL * g.rows * g.h;
    pmax = std::max(pmax, (long long)fwd_a2_blocks(g));
    c->g.push_back(g);
  }
  c->ntot = vox;
  c->nspec = spec;
  c->pstride = pmax;
  // twiddle tables, one per distinct axis length
  for (auto& g : c->g)
    for (int d = 0; d < 3; ++d) {
      const int n = g.ax[d].n;
      auto it = std::find(c->tw_len.begin(), c->tw_len.end(), n);
      if (it == c->tw_len.end()) {
        c->tw_len.push_back(n);
        c->tw_off.push_back(c->tw_total);
        g.ax[d].tw = c->tw_total;
        c->tw_total += n;
      } else {
        g.ax[d].tw = c->tw_off[it - c->tw_len.begin()];
      }
    }
  // workspace layout
  const size_t f64 = 9 * (size_t)vox * sizeof(double);
  const size_t fv = 9 * (size_t)vox * (c->prec == PREC_F64 ? 8 : 4);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  c->o_Ft = take(f64);
  c->o_F = take(f64);
  c->o_P = take(f64);
  c->o_x = take(fv);
  c->o_r = take(fv);
  c->o_p = take(fv);
  c->o_w = take(fv);
  c->o_F32 = take(c->prec == PREC_F32 ? 9 * (size_t)vox * 4 : 0);
  c->o_spec = take((size_t)spec * 16);
  c->o_phase = take((size_t)vox);
  c->o_mu = take((size_t)vox * 8);
  c->o_mtab = take(kMaxPhase * 4 * 8);
  c->o_part = take((size_t)NSLOT * pmax * 8);
  c->o_cg = take((size_t)nrve * sizeof(CgState));
  c->o_red = take((size_t)NSLOT * 8);
  c->o_tw64 = take((size_t)c->tw_total * 16);
  c->o_tw32 = take((size_t)c->tw_total * 8);
  c->total = o;
  c->Fbar_t.assign(9 * (size_t)nrve, 0.0);
  if (hipHostMalloc(reinterpret_cast<void**>(&c->pinned), 4096) != hipSuccess) return FFTNK_EHIP;
  return FFTNK_OK;
}

int reset_state(fftnk_ctx* c) {
  for (int r = 0; r < c->nrve; ++r) {
    launch_set_identity(c->args(r), c->Ft(), c->stream);
    for (int k = 0; k < 9; ++k) c->Fbar_t[9 * r + k] = (k % 4 == 0) ? 1.0 : 0.0;
  }
  int e = check_launch();
  if (e) return e;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return FFTNK_OK;
}

// ---------------------------------------------------------------------------
// the five passes of one projection G( Y ) where Y is produced by the first
// pass according to `mode`
// ---------------------------------------------------------------------------
void middle_passes(fftnk_ctx* c, int prec, const PassArgs& a, const CgState* cg) {
  launch_col_a1(prec, false, a, c->spec(), cg, c->stream);
  launch_col_a0_project(prec, a, c->spec(), cg, c->stream);
  launch_col_a1(prec, true, a, c->spec(), cg, c->stream);
}

// b = -G(Y) in FP64, written to r (context precision) with x = 0;
// partials: ||Y||^2 in SLOT_YY, ||b||^2 in SLOT_BB.
void rhs_pipeline(fftnk_ctx* c, int r, int mode, const double* Y, const double* Flin, const double* uni,
                  double sign = -1.0) {
  const PassArgs a = c->args(r);
  const Material m = c->material();
  launch_fwd_a2(PREC_F64, mode, a, m, Y, nullptr, nullptr, Flin, uni, 1.0, c->spec(), nullptr, c->stream);
  middle_passes(c, PREC_F64, a, nullptr);
  launch_inv_a2(PREC_F64, INV_RHS, a, c->spec(), c->r(), c->prec, nullptr, c->x(), sign, nullptr, c->stream);
}

// CG on A = G K(Flin) with right-hand side r (x = 0 on entry).
int run_cg(fftnk_ctx* c, int r, const void* Flin, double eta, int max_cg, int* iters, double* relres) {
  const PassArgs a = c->args(r);
  const Material m = c->material();
  CgState* cg = c->cg(r);
  const int stall = c->prec == PREC_F32 ? 50 : 0;
  launch_cg_init(a, inv_a2_blocks(a.g), cg, eta, max_cg, stall, c->stream);
  int launched = 0, chunk = 4;
  while (true) {
    for (int k = 0; k < chunk; ++k) {
      launch_fwd_a2(c->prec, FWD_CG, a, m, nullptr, c->r(), c->p(), Flin, nullptr, 1.0, c->spec(), cg, c->stream);
      middle_passes(c, c->prec, a, cg);
      launch_inv_a2(c->prec, INV_PW, a, c->spec(), c->w(), c->prec, c->p(), nullptr, 1.0, cg, c->stream);
      launch_cg_alpha(a, inv_a2_blocks(a.g), cg, c->stream);
      launch_cg_update(c->prec, a, c->x(), c->r(), c->p(), c->w(), cg, c->stream);
      launch_cg_beta(a, cg, c->stream);
    }
    launched += chunk;
    int st = check_launch();
    if (st) return st;
    st = fetch(c, cg, sizeof(CgState));
    if (st) return st;
    CgState h;
    std::memcpy(&h, c->pinned, sizeof(h));
    if (h.done) {
      *iters = h.iter;
      *relres = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
      return h.status;  // kernel status values equal the FFTNK_* codes
    }
    if (launched > max_cg + 64) return FFTNK_ECG_MAXIT;  // unreachable: k_cg_beta stops at max_cg
    chunk = std::min(chunk * 2, 32);
  }
}

int solve_rve(fftnk_ctx* c, int r, const double* Fbar, double eta_nw, double eta_cg, int max_newton, int max_cg,
              fftnk_stats* st) {
  const PassArgs a = c->args(r);
  const Grid& g = a.g;
  const Material m = c->material();
  const hipStream_t s = c->stream;
  double* red = c->red();
  const int nvox = elem_blocks_vox(g);
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(Fbar[k])) return FFTNK_ENONFINITE;

  // dFbar = Fbar - mean(F_t)  (Sec. 3.1)
  launch_field_sum(a, c->Ft(), SLOT_FBAR, s);
  launch_reduce(a, SLOT_FBAR, 9, nvox, red, s);
  int e = check_launch();
  if (!e) e = fetch(c, red, 9 * sizeof(double));
  if (e) return e;
  double dFbar[9];
  for (int k = 0; k < 9; ++k) dFbar[k] = Fbar[k] - c->pinned[k] / (double)g.n;

  // boundary-condition right-hand side with the tangent of the start state
  rhs_pipeline(c, r, FWD_TANGENT_UNI, nullptr, c->Ft(), dFbar);
  launch_set_F(a, c->Ft(), c->F(), dFbar, c->F32(), s);
  launch_reduce(a, SLOT_YY, 1, fwd_a2_blocks(g), red + 0, s);
  launch_reduce(a, SLOT_BB, 1, inv_a2_blocks(g), red + 1, s);
  launch_reduce(a, SLOT_FF, 1, nvox, red + 2, s);
  e = check_launch();
  if (!e) e = fetch(c, red, 3 * sizeof(double));
  if (e) return e;
  double yy = c->pinned[0], bb = c->pinned[1];
  const double Fn = std::sqrt(c->pinned[2]);

  const double eta_eff = c->prec == PREC_F32 ? std::max(eta_cg, 1e-6) : eta_cg;
  for (int it = 0;; ++it) {
    if (it >= max_newton) return FFTNK_ENEWTON_MAXIT;
    int iters = 0;
    double relres = 0.0;
    if (!std::isfinite(bb) || !std::isfinite(yy)) return FFTNK_ENONFINITE;
    if (!(std::sqrt(bb) <= 1e-14 * std::sqrt(yy) || bb == 0.0)) {
      const void* Flin = c->prec == PREC_F32 ? static_cast<const void*>(c->F32())
                                             : static_cast<const void*>(it == 0 ? c->Ft() : c->F());
      e = run_cg(c, r, Flin, eta_eff, max_cg, &iters, &relres);
      if (st) {
        st->cg_iters[it] = iters;
        st->cg_relres[it] = relres;
        st->n_solves = it + 1;
      }
      if (e) return e;
    } else if (st) {
      st->cg_iters[it] = 0;
      st->cg_relres[it] = 0.0;
      st->n_solves = it + 1;
    }
    // F += dF, constitutive update, new right-hand side -G(P)
    launch_newton_update(c->prec, a, m, c->F(), c->x(), c->P(), c->F32(), s);
    rhs_pipeline(c, r, FWD_COPY, c->P(), nullptr, nullptr);
    launch_reduce(a, SLOT_DF, 1, nvox, red + 0, s);
    launch_reduce(a, SLOT_PBAR, 9, nvox, red + 1, s);
    launch_reduce(a, SLOT_YY, 1, fwd_a2_blocks(g), red + 10, s);
    launch_reduce(a, SLOT_BB, 1, inv_a2_blocks(g), red + 11, s);
    e = check_launch();
    if (!e) e = fetch(c, red, 12 * sizeof(double));
    if (e) return e;
    const double df = c->pinned[0];
    yy = c->pinned[10];
    bb = c->pinned[11];
    const double res = std::sqrt(df) / Fn;
    if (st) st->newton_res[it] = res;
    if (!std::isfinite(res)) return FFTNK_ENONFINITE;
    for (int k = 0; k < 9; ++k)
      if (!std::isfinite(c->pinned[1 + k])) return FFTNK_ENONFINITE;
    if (res < eta_nw && it > 0) break;
  }
  // converged: P-bar, commit F_t
  for (int k = 0; k < 9; ++k) c->Fbar_t[9 * r + k] = Fbar[k];
  return FFTNK_OK;
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================
extern "C" {

int fftnk_create(fftnk_ctx** out, int n0, int n1, int n2, int precision, void* hip_stream) {
  const int dims[3] = {n0, n1, n2};
  return fftnk_create_batched(out, 1, dims, precision, hip_stream);
}

int fftnk_create_batched(fftnk_ctx** out, int nrve, const int* dims, int precision, void* hip_stream) {
  if (!out) return FFTNK_EINVAL;
  *out = nullptr;
  fftnk_ctx* c = new (std::nothrow) fftnk_ctx();
  if (!c) return FFTNK_EINVAL;
  const int e = init_ctx(c, nrve, dims, precision, hip_stream);
  if (e) {
    fftnk_destroy(c);
    return e;
  }
  *out = c;
  return FFTNK_OK;
}

size_t fftnk_workspace_bytes(const fftnk_ctx* c) { return c ? c->total : 0; }

int fftnk_bind_workspace(fftnk_ctx* c, void* dev, size_t bytes) {
  if (!c || !dev) return FFTNK_EINVAL;
  if ((reinterpret_cast<uintptr_t>(dev) % kAlign) != 0) return FFTNK_EINVAL;
  if (bytes < c->total) return FFTNK_ENOMEM;
  c->ws = static_cast<char*>(dev);
  // twiddle tables W_n^e = exp(-2 pi i e / n), FP64 and FP32
  std::vector<double> t64(2 * (size_t)c->tw_total);
  std::vector<float> t32(2 * (size_t)c->tw_total);
  const double two_pi = 6.283185307179586476925286766559;
  for (size_t i = 0; i < c->tw_len.size(); ++i) {
    const int n = c->tw_len[i];
    for (int e = 0; e < n; ++e) {
      const double ang = -two_pi * (double)e / (double)n;
      const size_t k = 2 * ((size_t)c->tw_off[i] + e);
      t64[k] = std::cos(ang);
      t64[k + 1] = std::sin(ang);
      t32[k] = (float)t64[k];
      t32[k + 1] = (float)t64[k + 1];
    }
  }
  HIP_TRY(hipMemcpyAsync(c->ws + c->o_tw64, t64.data(), t64.size() * 8, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->ws + c->o_tw32, t32.data(), t32.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemsetAsync(c->ws + c->o_cg, 0, (size_t)c->nrve * sizeof(CgState), c->stream));
  HIP_TRY(hipMemsetAsync(c->ws + c->o_part, 0, (size_t)NSLOT * c->pstride * 8, c->stream));
  return reset_state(c);
}

int fftnk_set_phases(fftnk_ctx* c, const uint8_t* phase_dev) {
  if (!c || !phase_dev) return FFTNK_EINVAL;
  if (!c->ws) return FFTNK_ESTATE;
  HIP_TRY(hipMemcpyAsync(c->ws + c->o_phase, phase_dev, (size_t)c->ntot, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->have_phase = true;
  return FFTNK_OK;
}

int fftnk_set_material(fftnk_ctx* c, int model, int nphase, const double* params) {
  if (!c || !params || nphase < 1 || nphase > kMaxPhase) return FFTNK_EINVAL;
  if (model != FFTNK_SVK) return FFTNK_EUNSUPPORTED;
  if (!c->ws) return FFTNK_ESTATE;
  const int np = model == FFTNK_SVK ? 2 : 4;
  for (int i = 0; i < nphase * np; ++i)
    if (!std::isfinite(params[i])) return FFTNK_EINVAL;
  std::memset(c->mtab, 0, sizeof(c->mtab));
  for (int ph = 0; ph < nphase; ++ph)
    for (int k = 0; k < np; ++k) c->mtab[4 * ph + k] = params[np * ph + k];
  c->model = model;
  c->nphase = nphase;
  HIP_TRY(hipMemcpyAsync(c->ws + c->o_mtab, c->mtab, sizeof(c->mtab), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->have_mat = true;
  return FFTNK_OK;
}

int fftnk_set_modulus_field(fftnk_ctx* c, const double* mu_dev) {
  if (!c) return FFTNK_EINVAL;
  if (!c->ws) return FFTNK_ESTATE;
  if (!mu_dev) {
    c->use_mu = false;
    return FFTNK_OK;
  }
  HIP_TRY(hipMemcpyAsync(c->ws + c->o_mu, mu_dev, (size_t)c->ntot * 8, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->use_mu = true;
  return FFTNK_OK;
}

int fftnk_reset_state(fftnk_ctx* c) {
  if (!c) return FFTNK_EINVAL;
  if (!c->ws) return FFTNK_ESTATE;
  return reset_state(c);
}

int fftnk_solve_increment(fftnk_ctx* c, const double* Fbar, double eta_nw, double eta_cg, int max_newton, int max_cg,
                          double* F_dev, double* P_dev, double* Pbar, fftnk_stats* stats) {
  if (!c || !Fbar || !Pbar) return FFTNK_EINVAL;
  if (!(eta_nw > 0) || !(eta_cg > 0) || max_newton < 2 || max_newton > FFTNK_MAX_SOLVES || max_cg < 1)
    return FFTNK_EINVAL;
  if (!c->ws || !c->have_phase || !c->have_mat) return FFTNK_ESTATE;
  const auto t0 = std::chrono::steady_clock::now();
  int worst = FFTNK_OK;
  std::vector<int> ok(c->nrve, 0);
  for (int r = 0; r < c->nrve; ++r) {
    fftnk_stats local;
    fftnk_stats* st = stats ? &stats[r] : &local;
    std::memset(st, 0, sizeof(*st));
    const int e = solve_rve(c, r, Fbar + 9 * r, eta_nw, eta_cg, max_newton, max_cg, st);
    st->status = e;
    if (e) {
      if (!worst) worst = e;
      continue;
    }
    ok[r] = 1;
    const Grid& g = c->g[r];
    const PassArgs a = c->args(r);
    launch_reduce(a, SLOT_PBAR, 9, elem_blocks_vox(g), c->red(), c->stream);
    int e2 = check_launch();
    if (!e2) e2 = fetch(c, c->red(), 9 * sizeof(double));
    if (e2) return e2;
    for (int k = 0; k < 9; ++k) Pbar[9 * r + k] = c->pinned[k] / (double)g.n;
  }
  // commit the converged RVEs (transactional per RVE), copy out
  const size_t f64 = 9 * (size_t)c->ntot * sizeof(double);
  for (int r = 0; r < c->nrve; ++r) {
    if (!ok[r]) continue;
    const Grid& g = c->g[r];
    const size_t off = 9 * (size_t)g.vox_off, bytes = 9 * (size_t)g.n * sizeof(double);
    HIP_TRY(hipMemcpyAsync(c->Ft() + off, c->F() + off, bytes, hipMemcpyDeviceToDevice, c->stream));
    if (F_dev) HIP_TRY(hipMemcpyAsync(F_dev + off, c->F() + off, bytes, hipMemcpyDeviceToDevice, c->stream));
    if (P_dev) HIP_TRY(hipMemcpyAsync(P_dev + off, c->P() + off, bytes, hipMemcpyDeviceToDevice, c->stream));
  }
  (void)f64;
  HIP_TRY(hipStreamSynchronize(c->stream));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats)
    for (int r = 0; r < c->nrve; ++r) stats[r].t_ms = ms;
  return worst;
}

int fftnk_set_linearization(fftnk_ctx* c, const double* F_dev) {
  if (!c || !F_dev) return FFTNK_EINVAL;
  if (!c->ws) return FFTNK_ESTATE;
  const size_t bytes = 9 * (size_t)c->ntot * sizeof(double);
  HIP_TRY(hipMemcpyAsync(c->F(), F_dev, bytes, hipMemcpyDeviceToDevice, c->stream));
  if (c->prec == PREC_F32) launch_convert(PREC_F32, c->F(), c->F32(), 9 * c->ntot, c->stream);
  HIP_TRY(hipStreamSynchronize(c->stream));
  return check_launch();
}

int fftnk_apply_operator(fftnk_ctx* c, const void* p_dev, void* Ap_dev) {
  if (!c || !p_dev || !Ap_dev || p_dev == Ap_dev) return FFTNK_EINVAL;
  if (!c->ws || !c->have_phase || !c->have_mat) return FFTNK_ESTATE;
  const Material m = c->material();
  const void* Flin = c->prec == PREC_F32 ? static_cast<const void*>(c->F32()) : static_cast<const void*>(c->F());
  for (int r = 0; r < c->nrve; ++r) {
    const PassArgs a = c->args(r);
    launch_fwd_a2(c->prec, FWD_TANGENT, a, m, p_dev, nullptr, nullptr, Flin, nullptr, 1.0, c->spec(), nullptr,
                  c->stream);
    middle_passes(c, c->prec, a, nullptr);
    launch_inv_a2(c->prec, INV_OUT, a, c->spec(), Ap_dev, c->prec, nullptr, nullptr, 1.0, nullptr, c->stream);
  }
  return check_launch();
}

int fftnk_adjoint(fftnk_ctx* c, const double* gbar, double eta_cg, int max_cg, double* dLdmu, double* dLdK,
                  fftnk_stats* stats) {
  if (!c || !gbar || !dLdmu || !(eta_cg > 0) || max_cg < 1) return FFTNK_EINVAL;
  if (!c->ws || !c->have_phase || !c->have_mat) return FFTNK_ESTATE;
  const size_t bytes = (size_t)c->ntot * sizeof(double);
  HIP_TRY(hipMemsetAsync(dLdmu, 0, bytes, c->stream));
  if (dLdK) HIP_TRY(hipMemsetAsync(dLdK, 0, bytes, c->stream));
  const double eta_eff = c->prec == PREC_F32 ? std::max(eta_cg, 1e-6) : eta_cg;
  int worst = FFTNK_OK;
  for (int r = 0; r < c->nrve; ++r) {
    const PassArgs a = c->args(r);
    const Grid& g = a.g;
    fftnk_stats local;
    fftnk_stats* st = stats ? &stats[r] : &local;
    std::memset(st, 0, sizeof(*st));
    for (int k = 0; k < 9; ++k)
      if (!std::isfinite(gbar[9 * r + k])) return FFTNK_ENONFINITE;
    // b = +G(K(F_t) : g), adjoint of the boundary-condition system
    rhs_pipeline(c, r, FWD_TANGENT_UNI, nullptr, c->Ft(), gbar + 9 * r, +1.0);
    if (c->prec == PREC_F32)
      launch_convert(PREC_F32, c->Ft() + 9 * g.vox_off, c->F32() + 9 * g.vox_off, 9 * g.n, c->stream);
    launch_reduce(a, SLOT_YY, 1, fwd_a2_blocks(g), c->red() + 0, c->stream);
    launch_reduce(a, SLOT_BB, 1, inv_a2_blocks(g), c->red() + 1, c->stream);
    int e = check_launch();
    if (!e) e = fetch(c, c->red(), 2 * sizeof(double));
    if (e) return e;
    const double yy = c->pinned[0], bb = c->pinned[1];
    int iters = 0;
    double relres = 0.0;
    if (!std::isfinite(bb)) return FFTNK_ENONFINITE;
    if (!(std::sqrt(bb) <= 1e-14 * std::sqrt(yy) || bb == 0.0)) {
      const void* Flin = c->prec == PREC_F32 ? static_cast<const void*>(c->F32()) : static_cast<const void*>(c->Ft());
      e = run_cg(c, r, Flin, eta_eff, max_cg, &iters, &relres);
    }
    st->n_solves = 1;
    st->cg_iters[0] = iters;
    st->cg_relres[0] = relres;
    st->status = e;
    if (e) {
      if (!worst) worst = e;
      continue;
    }
    launch_adjoint_grad(c->prec, a, c->Ft(), c->x(), gbar + 9 * r, dLdmu, dLdK, g.vox_off, c->stream);
  }
  const int e = check_launch();
  HIP_TRY(hipStreamSynchronize(c->stream));
  return worst ? worst : e;
}

int fftnk_launch_pass(fftnk_ctx* c, int pass) {
  if (!c || pass < 1 || pass > 5) return FFTNK_EINVAL;
  if (!c->ws || !c->have_phase || !c->have_mat) return FFTNK_ESTATE;
  const Material m = c->material();
  const void* Flin = c->prec == PREC_F32 ? static_cast<const void*>(c->F32()) : static_cast<const void*>(c->F());
  for (int r = 0; r < c->nrve; ++r) {
    const PassArgs a = c->args(r);
    switch (pass) {
      case 1:
        launch_fwd_a2(c->prec, FWD_TANGENT, a, m, c->p(), nullptr, nullptr, Flin, nullptr, 1.0, c->spec(), nullptr,
                      c->stream);
        break;
      case 2: launch_col_a1(c->prec, false, a, c->spec(), nullptr, c->stream); break;
      case 3: launch_col_a0_project(c->prec, a, c->spec(), nullptr, c->stream); break;
      case 4: launch_col_a1(c->prec, true, a, c->spec(), nullptr, c->stream); break;
      default:
        launch_inv_a2(c->prec, INV_OUT, a, c->spec(), c->w(), c->prec, nullptr, nullptr, 1.0, nullptr, c->stream);
        break;
    }
  }
  return check_launch();
}

int fftnk_project(fftnk_ctx* c, const void* a_dev, void* Ga_dev) {
  if (!c || !a_dev || !Ga_dev) return FFTNK_EINVAL;
  if (!c->ws) return FFTNK_ESTATE;
  const Material m = c->material();
  for (int r = 0; r < c->nrve; ++r) {
    const PassArgs a = c->args(r);
    launch_fwd_a2(c->prec, FWD_COPY, a, m, a_dev, nullptr, nullptr, nullptr, nullptr, 1.0, c->spec(), nullptr,
                  c->stream);
    middle_passes(c, c->prec, a, nullptr);
    launch_inv_a2(c->prec, INV_OUT, a, c->spec(), Ga_dev, c->prec, nullptr, nullptr, 1.0, nullptr, c->stream);
  }
  return check_launch();
}

int fftnk_constitutive(fftnk_ctx* c, const double* F_dev, double* P_dev, double* Pbar) {
  if (!c || !F_dev || !P_dev || !Pbar) return FFTNK_EINVAL;
  if (!c->ws || !c->have_phase || !c->have_mat) return FFTNK_ESTATE;
  const Material m = c->material();
  for (int r = 0; r < c->nrve; ++r) {
    const PassArgs a = c->args(r);
    launch_constitutive(a, m, F_dev, P_dev, c->stream);
    launch_reduce(a, SLOT_PBAR, 9, elem_blocks_vox(a.g), c->red(), c->stream);
    int e = check_launch();
    if (!e) e = fetch(c, c->red(), 9 * sizeof(double));
    if (e) return e;
    for (int k = 0; k < 9; ++k) Pbar[9 * r + k] = c->pinned[k] / (double)a.g.n;
  }
  return FFTNK_OK;
}

int fftnk_get_state(fftnk_ctx* c, double* F_dev) {
  if (!c || !F_dev) return FFTNK_EINVAL;
  if (!c->ws) return FFTNK_ESTATE;
  HIP_TRY(hipMemcpyAsync(F_dev, c->Ft(), 9 * (size_t)c->ntot * 8, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return FFTNK_OK;
}

int fftnk_set_state(fftnk_ctx* c, const double* F_dev) {
  if (!c || !F_dev) return FFTNK_EINVAL;
  if (!c->ws) return FFTNK_ESTATE;
  HIP_TRY(hipMemcpyAsync(c->Ft(), F_dev, 9 * (size_t)c->ntot * 8, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return FFTNK_OK;
}

const char* fftnk_status_string(int s) {
  switch (s) {
    case FFTNK_OK: return "ok";
    case FFTNK_EINVAL: return "invalid argument";
    case FFTNK_ESTATE: return "call order (workspace, phases or material not set)";
    case FFTNK_ENOMEM: return "workspace too small";
    case FFTNK_EHIP: return "HIP runtime error";
    case FFTNK_ECG_MAXIT: return "CG iteration limit reached";
    case FFTNK_ECG_BREAKDOWN: return "CG breakdown (indefinite or non-finite <p, Ap>)";
    case FFTNK_ENEWTON_MAXIT: return "Newton iteration limit reached";
    case FFTNK_ENONFINITE: return "non-finite value";
    case FFTNK_EMATERIAL: return "constitutive update failed";
    case FFTNK_EUNSUPPORTED: return "unsupported size or configuration";
    default: return "unknown status";
  }
}

void fftnk_destroy(fftnk_ctx* c) {
  if (!c) return;
  if (c->pinned) (void)hipHostFree(c->pinned);
  delete c;
}

}  // extern "C"
