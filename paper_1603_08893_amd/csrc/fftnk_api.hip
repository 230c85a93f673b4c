// Host driver and C-ABI of libfftnk (declared in include/fftnk.h).
//
// The driver runs Algorithm 1 of de Geus et al. (2017) for one load increment
// on every RVE of a context at once: boundary-condition solve with the tangent
// of the start state (Sec. 3.1), Newton iterations on G:K:dF = -G:P (Sec. 2.6)
// each solved by CG, the convergence test ||dF|| / ||F_t + dFbar|| < eta_NW
// after at least two solves, and the transactional commit of the converged
// state ("store converged state", Alg. 1).  All field work runs in the kernels
// (fftnk_fft_kernels.hip, fftnk_solver_kernels.hip); every launch covers all
// RVEs, finished RVEs are masked on the device.  CG iterations are replayed
// from captured HIP graphs; the host reads back a few scalars per Newton
// iteration and per batch of CG iterations.
#include "fftnk.h"
#include "fftnk_internal.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace fftnk;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Radix plan: primes of 11 and above first, largest first (the first stage
// has no stage twiddles, and a prime stage would otherwise apply them once per
// group of output pairs), then the power-of-two part in as few stages of
// 8 / 4 / 2 as possible (bits spread evenly), then 3, 5, 7.
bool make_plan(int n, AxisPlan& pl, bool allow12) {
  pl.n = n;
  pl.nstages = 0;
  int m = n, e2 = 0;
  {
    int big[kMaxStages], nb = 0, r = n;
    for (int p = 2; p * p <= r; ++p)
      while (r % p == 0) {
        if (p >= 11) big[nb++] = p;
        r /= p;
      }
    if (r >= 11) big[nb++] = r;
    for (int i = nb - 1; i >= 0; --i) {  // ascending factorisation: largest last
      if (pl.nstages >= kMaxStages) return false;
      pl.radix[pl.nstages++] = big[i];
      m /= big[i];
    }
  }
  while (m % 2 == 0) {
    m /= 2;
    ++e2;
  }
  if (e2 > 0) {
    const int ns = (e2 + 2) / 3;
    std::vector<int> b(ns, e2 / ns);
    for (int s = 0; s < e2 % ns; ++s) b[s] += 1;
    for (int s = 0; s < ns; ++s) {
      if (pl.nstages >= kMaxStages) return false;
      pl.radix[pl.nstages++] = 1 << b[s];
    }
  }
  for (int p = 3; m > 1 && p <= 7; p += 2) {
    while (m % p == 0) {
      if (pl.nstages >= kMaxStages) return false;
      pl.radix[pl.nstages++] = p;
      m /= p;
    }
  }
  if (m != 1) return false;
  if ((1 << e2) == n && e2 >= 3 && n <= kMaxRegLen)
    pl.reg = 8;
  else if (allow12 && n == 3 * (1 << e2) && e2 >= 2 && n <= 192)
    pl.reg = 12;
  else
    pl.reg = 0;
  return true;
}

// pencils per work-group in the LDS-engine a1 / a0 passes (consecutive in
// the spectrum's k2-fastest order, so runs of at least 128 bytes where
// possible), within the LDS (60 KiB) and register (kMaxPpt points per thread
// in pass 3) budgets.
int pick_m(int nmax, size_t csz, int pref) {
  int m = pref;
  while (m > 1 && ((size_t)nmax * m > (size_t)kMaxPpt * kThreads || csz * ((size_t)padded_len(nmax) + 2 * (size_t)nmax * m) > 61440))
    m /= 2;
  return m;
}

// a2 passes: twiddles + pencil buffers for `rt` lines (5 pencils each): one
// padded slot per pencil plus one spare slot shared by the idle pencil slots
// (register engine), or two ping-pong buffers (LDS engine)
size_t row_lds(const Grid& g, int rt, int engine, size_t csz) {
  const size_t tw = padded_len(g.n2);
  if (engine) return csz * (tw + (5 * (size_t)rt + 1) * padded_len(g.n2));
  return csz * (tw + 2 * 5 * (size_t)rt * g.n2);
}
size_t col_lds(const Grid& g, int axis, size_t csz) {
  const int n = axis == 0 ? g.n0 : g.n1;
  if (g.ax[axis].reg) return csz * ((size_t)padded_len(n) + (size_t)kThreads * g.ax[axis].reg);
  const int M = csz == 16 ? g.m64 : g.m32;
  return csz * ((size_t)padded_len(n) + 2 * (size_t)n * M);
}

// Plan policy (fftnk_set_plan): bits 0-2, axis d on the LDS engine even where
// a register engine exists; bits 3-4, s <= 2: the LDS-engine column passes
// take at most 8 >> s (FP64) / 16 >> s (FP32) pencils per work-group; bit 5,
// the register-engine a2 passes take half their default grid lines per
// work-group.  Every policy computes the same transforms; only engines and
// tile sizes differ.
constexpr unsigned kPolicyCodes = 64;
bool policy_valid(unsigned pol) { return pol < kPolicyCodes && ((pol >> 3) & 3u) != 3u; }

// engines and tile sizes of one cell under `pol` (radix plans and twiddle
// offsets stay)
void plan_cell(Grid& g, unsigned pol) {
  for (int d = 0; d < 3; ++d) {
    AxisPlan& a = g.ax[d];
    const int tw = a.tw;
    make_plan(a.n, a, true);
    a.tw = tw;
    if (pol & (1u << d)) a.reg = 0;
  }
  // grid lines per a2 work-group: register engine, 5 pair pencils per line on
  // kThreads / (n2/P) pencil slots, within 48 KiB of FP64 LDS (5 rt pencils +
  // one spare slot: three work-groups per CU at least); LDS engine, kThreads / n2
  if (g.ax[2].reg) {
    const int slots = kThreads / (g.n2 / g.ax[2].reg);
    const int fit = (49152 / 16 - padded_len(g.n2)) / padded_len(g.n2) - 1;
    g.rt = std::max(1, std::min(slots / 5, fit / 5));
    if (pol & 32u) g.rt = std::max(1, g.rt / 2);
  } else {
    g.rt = std::max(1, kThreads / g.n2);
  }
  // forward pass: at most one voxel per thread in its tangent phase, so that
  // all loads of a work-group are in flight together (and the register-engine
  // line count, or kThreads / n2 on the LDS engine)
  g.rt1 = pass1_engine(g.ax[2].reg) ? std::max(1, std::min(g.rt, kThreads / g.n2)) : std::max(1, kThreads / g.n2);
  const int nmax = std::max(g.n0, g.n1);
  const int s = (int)((pol >> 3) & 3u);
  g.m64 = pick_m(nmax, 16, 8 >> s);
  g.m32 = pick_m(nmax, 8, 16 >> s);
}

// launch geometry of a context's cells under one policy
struct Geo {
  std::vector<Grid> g;
  std::vector<int> starts;  // [NKIND][nrve + 1]
  int nblk[NKIND] = {};
  size_t lds[8] = {};
  int eng[3] = {};
  long long pstride = 0;  // most work-groups of any launch kind
};

// EUNSUPPORTED when a kernel's LDS budget or the work-group count is exceeded
int make_geo(const std::vector<Grid>& cells, unsigned pol, Geo& o) {
  const int nrve = (int)cells.size();
  o.g = cells;
  for (Grid& g : o.g) plan_cell(g, pol);
  o.starts.assign((size_t)NKIND * (nrve + 1), 0);
  for (int k = 0; k < NKIND; ++k) {
    long long acc = 0;
    for (int r = 0; r < nrve; ++r) {
      const Grid& g = o.g[r];
      o.starts[k * (nrve + 1) + r] = (int)acc;
      long long b = 0;
      switch (k) {
        case K_ROW: b = row_blocks(g); break;
        case K_ROW1: b = row1_blocks(g); break;
        case K_COL1_64: b = col1_blocks(g, PREC_F64); break;
        case K_COL1_32: b = col1_blocks(g, PREC_F32); break;
        case K_COL0_64: b = col0_blocks(g, PREC_F64); break;
        case K_COL0_32: b = col0_blocks(g, PREC_F32); break;
        case K_ELEM9: b = elem_blocks(9 * g.n); break;
        default: b = elem_blocks(g.n); break;
      }
      acc += b;
    }
    if (acc > (1LL << 30)) return FFTNK_EUNSUPPORTED;
    o.starts[k * (nrve + 1) + nrve] = (int)acc;
    o.nblk[k] = (int)acc;
    o.pstride = std::max(o.pstride, acc);
  }
  for (const Grid& g : o.g) {
    o.lds[0] = std::max(o.lds[0], row_lds(g, g.rt, g.ax[2].reg, 16));
    o.lds[1] = std::max(o.lds[1], row_lds(g, g.rt, g.ax[2].reg, 8));
    for (int d = 0; d < 3; ++d) {
      const bool pairs = d < 2 && col_engine(g.ax[d].reg, g.ax[d].n, g.h, g.spec_off, 4) == 16;
      o.eng[d] |= pairs ? 8 : g.ax[d].reg == 8 ? 2 : (g.ax[d].reg == 12 ? 4 : 1);
    }
    o.lds[6] = std::max(o.lds[6], row_lds(g, g.rt1, pass1_engine(g.ax[2].reg), 16));
    o.lds[7] = std::max(o.lds[7], row_lds(g, g.rt1, pass1_engine(g.ax[2].reg), 8));
    o.lds[2] = std::max(o.lds[2], col_lds(g, 1, 16));
    o.lds[3] = std::max(o.lds[3], col_lds(g, 1, 8));
    o.lds[4] = std::max(o.lds[4], col_lds(g, 0, 16));
    o.lds[5] = std::max(o.lds[5], col_lds(g, 0, 8));
  }
  for (size_t b : o.lds)
    if (b > 61440) return FFTNK_EUNSUPPORTED;
  return FFTNK_OK;
}

}  // namespace

struct fftnk_ctx {
  int nrve = 0;
  int prec = PREC_F64;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;  // capture stream of the CG graphs
  std::vector<Grid> g;
  long long ntot = 0, nspec = 0;
  long long pstride = 0;  // partial-sum slot stride: the most work-groups of any launch kind under any policy
  std::vector<int> tw_len, tw_off;
  int tw_total = 0;
  std::vector<int> starts_full;  // [NKIND][nrve + 1] work-group ranges of every cell
  int nblk_full[NKIND] = {};
  std::vector<int> starts;  // the ranges launches use: those of the cells in the mask (compact_starts)
  int nblk[NKIND] = {};
  std::vector<int> graph_active;  // the mask the CG graphs were captured under
  size_t lds[8] = {};  // row64, row32, col1_64, col1_32, col0_64, col0_32, row1_64, row1_32
  int eng[3] = {};     // per axis: bit 0 some cell on the LDS engine, bit 1 on the 8-point, bit 2 on the 12-point one,
                       // bit 3 on the 8-point one with FP32 pencil pairs
  int nyq_id = 0;      // FFTNK_OPT_NYQUIST
  unsigned policy = 0;  // fftnk_set_plan
  int krylov = KRYLOV_CG;  // fftnk_set_krylov
  double k_lo = 0.0, k_hi = 0.0;
  int gm = 0;              // GMRES restart length (FFTNK_OPT_GMRES_RESTART), basis of gm + 1 vectors
  int jt = 0;              // FFTNK_OPT_J2_TANGENT: 1 = compact J2 tangent stored per linearisation point
  bool jt_ready = false;   // the stored compact tangent was computed (for the last linearisation point)
  size_t o_jt = 0;         // its workspace offset, [kJ2Tan][ntot] doubles after the GMRES basis
  int xwin = kMaxXWin;     // FFTNK_OPT_X_WINDOW: CG directions kept for the windowed x update
  size_t o_pwin = 0;       // their slots after the compact tangent (xwin > 1; else the p vector)
  size_t total_base = 0;   // workspace bytes without the GMRES basis
  // workspace layout (byte offsets)
  size_t o_hist, o_hnew;  // J2 history: committed and of the current iterate, [7][ntot] each
  size_t o_Ft, o_F, o_P, o_x, o_r, o_p, o_w, o_F32, o_d64, o_spec, o_phase, o_mu, o_mtab, o_part, o_cg, o_red,
      o_tw64, o_tw32, o_grids, o_starts, o_active, o_uni, o_nyq, o_coef, o_gm, total = 0;
  long long rows_total = 0;
  char* ws = nullptr;
  bool have_phase = false, have_mat = false, use_mu = false;
  int model = MODEL_SVK, nphase = 0;
  double mtab[kMaxPhase * 4] = {};
  unsigned char* pinned = nullptr;  // host staging for device -> host scalars
  size_t pinned_bytes = 0;
  std::vector<int> active;   // host copy of the Newton mask (uploaded when it changes)
  std::vector<double> uni;   // host copy of the per-RVE uniform tensors
  bool use_graphs = true;
  int check_every = 4;
  int cg_estimate = 8;
  std::map<int, hipGraphExec_t> graphs;

  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(ws + off);
  }
  double* Ft() const { return at<double>(o_Ft); }
  double* F() const { return at<double>(o_F); }
  double* P() const { return at<double>(o_P); }
  void* x() const { return ws + o_x; }
  void* r() const { return ws + o_r; }
  void* p() const { return ws + o_p; }
  // slot 0 of the CG directions (the others follow, pslot_bytes apart)
  void* pw() const { return ws + (xwin > 1 ? o_pwin : o_p); }
  size_t pslot_bytes() const { return align_up(9 * (size_t)ntot * (prec == PREC_F64 ? 8 : 4)); }
  void* w() const { return ws + o_w; }
  float* F32() const { return prec == PREC_F32 ? at<float>(o_F32) : nullptr; }
  double* d64() const { return at<double>(o_d64); }  // FP64 copy of the FP32 solution (FP32 mode)
  void* spec() const { return ws + o_spec; }
  CgState* cg() const { return at<CgState>(o_cg); }
  double* red() const { return at<double>(o_red); }
  // linearisation point of the CG kernels: F itself (FP64) or its FP32 copy
  const void* flin() const { return prec == PREC_F32 ? static_cast<const void*>(F32()) : static_cast<const void*>(F()); }

  Launch launch(hipStream_t s) const {
    Launch L;
    L.b.grids = at<Grid>(o_grids);
    L.b.starts = at<int>(o_starts);
    L.b.active = at<int>(o_active);
    L.b.uni = at<double>(o_uni);
    L.b.tw64 = ws + o_tw64;
    L.b.tw32 = ws + o_tw32;
    L.b.partials = at<double>(o_part);
    L.b.pstride = pstride;
    L.b.nyq = ws + o_nyq;
    L.b.nrve = nrve;
    L.b.xwin = xwin;
    L.b.vstride = (long long)(pslot_bytes() / (prec == PREC_F64 ? 8 : 4));
    for (int k = 0; k < NKIND; ++k) L.nblk[k] = nblk[k];
    L.lds_row64 = lds[0];
    L.lds_row32 = lds[1];
    L.lds_col1_64 = lds[2];
    L.lds_col1_32 = lds[3];
    L.lds_col0_64 = lds[4];
    L.lds_col0_32 = lds[5];
    L.lds_row1_64 = lds[6];
    L.lds_row1_32 = lds[7];
    for (int d = 0; d < 3; ++d) L.eng[d] = eng[d];
    L.nyq = nyq_id;
    L.ntop = op_nontemporal(ntot, prec == PREC_F64 ? 8 : 4);
    L.s = s;
    return L;
  }
  Launch launch() const { return launch(stream); }
  Material material() const {
    Material m;
    m.phase = at<uint8_t>(o_phase);
    m.mu_field = use_mu ? at<double>(o_mu) : nullptr;
    m.table = at<double>(o_mtab);
    m.hist = at<double>(o_hist);
    m.hist_new = at<double>(o_hnew);
    m.j2t = (jt_active() && jt_ready) ? at<double>(o_jt) : nullptr;
    m.ntot = ntot;
    m.model = model;
    m.nphase = nphase;
    return m;
  }
  bool jt_active() const { return jt && model == MODEL_J2 && prec == PREC_F64; }
  const CgState* host_cg() const { return reinterpret_cast<const CgState*>(pinned); }
  const double* host_red() const { return reinterpret_cast<const double*>(pinned); }
};

namespace {

// A named range on the host timeline (rocprofv3 --marker-trace) for the scope
// of one host-driver step; free when no profiler is attached.
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

#define HIP_TRY(expr)                            \
  do {                                           \
    if ((expr) != hipSuccess) return FFTNK_EHIP; \
  } while (0)

int check_launch() { return hipGetLastError() == hipSuccess ? FFTNK_OK : FFTNK_EHIP; }

int fetch(fftnk_ctx* c, const void* dev, size_t bytes) {
  if (bytes > c->pinned_bytes) return FFTNK_EINVAL;
  HIP_TRY(hipMemcpyAsync(c->pinned, dev, bytes, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return FFTNK_OK;
}

void compact_starts(fftnk_ctx* c);

// host arrays uploaded here stay untouched until the next stream synchronisation
// the Newton mask and the launch tables of its cells; every Launch built
// before this call is stale (its work-group counts)
int upload_active(fftnk_ctx* c) {
  compact_starts(c);
  HIP_TRY(hipMemcpyAsync(c->ws + c->o_active, c->active.data(), c->nrve * sizeof(int), hipMemcpyHostToDevice,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(c->ws + c->o_starts, c->starts.data(), c->starts.size() * sizeof(int),
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));  // the host tables may change again at once
  return FFTNK_OK;
}
// workspace bytes: the base layout, the GMRES basis, the compact J2 tangent
void size_workspace(fftnk_ctx* c) {
  size_t o = c->total_base;
  if (c->gm) o = align_up(o + (size_t)(c->gm + 1) * gm_vstride(c->ntot) * (c->prec == PREC_F64 ? 8 : 4));
  c->o_jt = o;
  if (c->jt) o = align_up(o + (size_t)kJ2Tan * c->ntot * sizeof(double));
  c->o_pwin = o;
  if (c->xwin > 1) o = align_up(o + (size_t)c->xwin * c->pslot_bytes());
  c->total = o;
}

// J2 with the stored tangent: the compact tangent at the linearisation point
// Flin (committed history), before a run of operator applications there
void refresh_j2_tangent(fftnk_ctx* c, const void* flin) {
  if (!c->jt_active()) return;
  launch_j2_tangent_data(c->launch(), c->material(), static_cast<const double*>(flin), c->at<double>(c->o_jt));
  c->jt_ready = true;
}

int upload_uni(fftnk_ctx* c) {
  HIP_TRY(hipMemcpyAsync(c->ws + c->o_uni, c->uni.data(), 9 * c->nrve * sizeof(double), hipMemcpyHostToDevice,
                         c->stream));
  return FFTNK_OK;
}

// Launch tables of the cells in the Newton mask: every other cell gets an
// empty work-group range, so a launch dispatches no work-group for it (cells
// that have finished their increment cost nothing); the full tables when all
// cells, or none, are in the mask.  Host side only.
void compact_starts(fftnk_ctx* c) {
  const int nr = c->nrve;
  int na = 0;
  for (int v : c->active) na += v != 0;
  c->starts = c->starts_full;
  std::copy(c->nblk_full, c->nblk_full + NKIND, c->nblk);
  if (na == 0 || na == nr || (int)c->active.size() != nr) return;
  for (int k = 0; k < NKIND; ++k) {
    const int* f = &c->starts_full[(size_t)k * (nr + 1)];
    int* t = &c->starts[(size_t)k * (nr + 1)];
    int acc = 0;
    for (int r = 0; r < nr; ++r) {
      t[r] = acc;
      if (c->active[r]) acc += f[r + 1] - f[r];
    }
    t[nr] = acc;
    c->nblk[k] = acc;
  }
}

void apply_geo(fftnk_ctx* c, const Geo& geo) {
  c->g = geo.g;
  c->starts_full = geo.starts;
  std::copy(geo.nblk, geo.nblk + NKIND, c->nblk_full);
  compact_starts(c);
  std::copy(geo.lds, geo.lds + 8, c->lds);
  std::copy(geo.eng, geo.eng + 3, c->eng);
}

int init_ctx(fftnk_ctx* c, int nrve, const int* dims, int precision, void* stream) {
  if (nrve < 1 || nrve > kMaxRve || !dims) return FFTNK_EINVAL;
  if (precision != FFTNK_FP64 && precision != FFTNK_FP32_MIXED) return FFTNK_EINVAL;
  c->nrve = nrve;
  c->prec = precision == FFTNK_FP64 ? PREC_F64 : PREC_F32;
  c->stream = static_cast<hipStream_t>(stream);
  long long vox = 0, spec = 0, rows = 0;
  for (int r = 0; r < nrve; ++r) {
    Grid g{};
    g.n0 = dims[3 * r];
    g.n1 = dims[3 * r + 1];
    g.n2 = dims[3 * r + 2];
    for (int d = 0; d < 3; ++d) {
      const int nd = dims[3 * r + d];
      const int lim = d == 2 ? kMaxLenA2 : kMaxLen;
      if (nd < 2 || nd > lim) return nd > lim ? FFTNK_EUNSUPPORTED : FFTNK_EINVAL;
      if (!make_plan(nd, g.ax[d], true)) return FFTNK_EUNSUPPORTED;
    }
    g.h = (g.n2 % 2 == 0) ? g.n2 / 2 : (g.n2 + 1) / 2;
    g.n = (long long)g.n0 * g.n1 * g.n2;
    g.rows = (long long)g.n0 * g.n1;
    g.vox_off = vox;
    g.spec_off = spec;
    g.row_off = rows;
    g.inv_n = 1.0 / (double)g.n;
    vox += g.n;
    spec += 9LL * g.rows * g.h;
    rows += g.rows;
    c->g.push_back(g);
  }
  c->ntot = vox;
  c->nspec = spec;
  c->rows_total = rows;
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
  // launch geometry under the default policy; the partial-sum slots are sized
  // for the largest launch of any policy
  Geo geo;
  int e = make_geo(c->g, 0, geo);
  if (e) return e;
  long long pmax = geo.pstride;
  for (unsigned pol = 1; pol < kPolicyCodes; ++pol) {
    Geo t;
    if (policy_valid(pol) && make_geo(c->g, pol, t) == FFTNK_OK) pmax = std::max(pmax, t.pstride);
  }
  apply_geo(c, geo);
  c->pstride = pmax;
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
  c->o_d64 = take(c->prec == PREC_F32 ? f64 : 0);
  c->o_spec = take((size_t)spec * 16);
  c->o_phase = take((size_t)vox);
  c->o_mu = take((size_t)vox * 8);
  c->o_hist = take((size_t)vox * 7 * 8);
  c->o_hnew = take((size_t)vox * 7 * 8);
  c->o_mtab = take(kMaxPhase * 4 * 8);
  c->o_part = take((size_t)NSLOT * c->pstride * 8);
  c->o_cg = take((size_t)nrve * sizeof(CgState));
  c->o_red = take((size_t)nrve * NSLOT * 8);
  c->o_tw64 = take((size_t)c->tw_total * 16);
  c->o_tw32 = take((size_t)c->tw_total * 8);
  c->o_grids = take((size_t)nrve * sizeof(Grid));
  c->o_starts = take(c->starts.size() * sizeof(int));
  c->o_active = take((size_t)nrve * sizeof(int));
  c->o_uni = take((size_t)nrve * 9 * sizeof(double));
  c->o_nyq = take(9 * (size_t)rows * sizeof(double));
  c->o_coef = take((size_t)nrve * kGmCoef * sizeof(double));
  c->o_gm = o;
  c->total_base = o;
  size_workspace(c);
  c->active.assign(nrve, 1);
  c->uni.assign(9 * (size_t)nrve, 0.0);
  c->pinned_bytes = std::max((size_t)nrve * NSLOT * 8, (size_t)nrve * sizeof(CgState)) + 256;
  return FFTNK_OK;  // no HIP call so far: the host staging and capture stream come with the workspace
}

void drop_graphs(fftnk_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

int reset_state(fftnk_ctx* c) {
  launch_set_identity(c->launch(), c->Ft());
  launch_set_virgin_history(c->launch(), c->at<double>(c->o_hist), c->ntot);
  int e = check_launch();
  if (e) return e;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return FFTNK_OK;
}

// ---------------------------------------------------------------------------
// pipelines
// ---------------------------------------------------------------------------
void middle_passes(int prec, const Launch& L, void* spec, const CgState* cg, CgState* alpha_cg = nullptr) {
  launch_col_a1(prec, false, L, spec, cg, alpha_cg);
  launch_col_a0_project(prec, L, spec, cg);
  launch_col_a1(prec, true, L, spec, cg);
}

// b = sign * G(Y) in FP64, written to r (context precision) with x = 0;
// partials: ||Y||^2 in SLOT_YY, ||b||^2 in SLOT_BB.  Y is produced by pass 1
// in `mode` (the field in, or the tangent at Flin applied to Batch::uni).
void rhs_pipeline(fftnk_ctx* c, int mode, const double* Y, const double* Flin, double sign) {
  const Range range_("fftnk right-hand side");
  if (mode != FWD_COPY) refresh_j2_tangent(c, Flin);
  const Launch L = c->launch();
  launch_fwd_a2(PREC_F64, mode, L, c->material(), Y, nullptr, nullptr, nullptr, Flin, 1.0, c->spec(), nullptr);
  middle_passes(PREC_F64, L, c->spec(), nullptr);
  launch_inv_a2(PREC_F64, INV_RHS, L, c->spec(), c->r(), c->prec, c->x(), sign, nullptr);
}

// The CG solution as the Newton update.  FP64: x itself.  FP32: x rounded up to
// FP64 and projected again with G in FP64.  In FP32 the Krylov vectors pick up
// rounding noise outside range(G) (incompatible and mean components) that the
// operator cannot see and the FP64 residual -G(P) can never remove; projecting
// the update restores compatibility and the prescribed mean exactly.
const void* newton_update_source(fftnk_ctx* c) {
  if (c->prec == PREC_F64) return c->x();
  const Launch L = c->launch();
  launch_convert(PREC_F64, c->x(), c->d64(), 9 * c->ntot, c->stream);
  launch_fwd_a2(PREC_F64, FWD_COPY, L, c->material(), c->d64(), nullptr, nullptr, nullptr, nullptr, 1.0, c->spec(),
                nullptr);
  middle_passes(PREC_F64, L, c->spec(), nullptr);
  launch_inv_a2(PREC_F64, INV_OUT, L, c->spec(), c->d64(), PREC_F64, nullptr, 1.0, nullptr);
  return c->d64();
}

// one CG iteration on every RVE whose CG is still running
void cg_iteration(fftnk_ctx* c, const Launch& L) {
  CgState* cg = c->cg();
  launch_fwd_a2(c->prec, FWD_CG, L, c->material(), nullptr, c->r(), c->pw(), c->x(), c->flin(), 1.0, c->spec(), cg);
  middle_passes(c->prec, L, c->spec(), cg, cg);  // alpha in extra work-groups of the a1 pass
  launch_inv_a2(c->prec, INV_CGR, L, c->spec(), c->r(), c->prec, nullptr, 1.0, cg);
  launch_cg_beta(L, cg);
}

// a HIP graph replaying k CG iterations (captured once per context)
int cg_graph(fftnk_ctx* c, int k, hipGraphExec_t* out) {
  auto it = c->graphs.find(k);
  if (it != c->graphs.end()) {
    *out = it->second;
    return FFTNK_OK;
  }
  HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  const Launch L = c->launch(c->cap);
  for (int i = 0; i < k; ++i) cg_iteration(c, L);
  hipGraph_t graph = nullptr;
  const hipError_t e1 = hipStreamEndCapture(c->cap, &graph);
  if (e1 != hipSuccess || !graph) return FFTNK_EHIP;
  hipGraphExec_t exec = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) return FFTNK_EHIP;
  c->graphs[k] = exec;
  *out = exec;
  return FFTNK_OK;
}

int launch_iterations(fftnk_ctx* c, int k, bool eager = false) {
  if (!c->use_graphs || eager) {
    const Launch L = c->launch();
    for (int i = 0; i < k; ++i) cg_iteration(c, L);
    return check_launch();
  }
  for (int chunk = 32; chunk >= 1; chunk /= 2) {
    while (k >= chunk) {
      hipGraphExec_t g = nullptr;
      const int e = cg_graph(c, chunk, &g);
      if (e) return e;
      HIP_TRY(hipGraphLaunch(g, c->stream));
      k -= chunk;
    }
  }
  return FFTNK_OK;
}

// CG on every active RVE: A = G K(linearisation point), right-hand side r,
// x = 0 on entry.  Per-RVE outcome in the device CgState array.
int run_gmres(fftnk_ctx* c, double eta, int max_it);

int run_cg(fftnk_ctx* c, double eta, int max_cg) {
  const Range range_("fftnk linear solve");
  refresh_j2_tangent(c, c->flin());
  if (c->krylov == KRYLOV_GMRES) return run_gmres(c, eta, max_cg);
  if (c->graph_active != c->active) {  // the graphs hold the launch sizes of another mask
    drop_graphs(c);
    c->graph_active = c->active;
  }
  const Launch L = c->launch();
  const int stall = c->prec == PREC_F32 ? 50 : 0;
  launch_cg_init(L, c->cg(), eta, max_cg, stall, c->krylov, c->k_lo, c->k_hi);
  int e = check_launch();
  if (e) return e;
  int launched = std::max(1, std::min(c->cg_estimate - 2, max_cg));
  e = launch_iterations(c, launched);
  if (e) return e;
  // Once some cells have finished their CG, the iterations that follow launch
  // over the others only: the mask is narrowed to the cells still iterating
  // (eager launches, the graphs keep the Newton mask's sizes) and the Newton
  // mask is restored before the last deferred x update, on every exit.
  struct Narrowed {
    fftnk_ctx* c;
    std::vector<int> newton;
    bool on = false;
    int restore() {
      if (!on) return FFTNK_OK;
      on = false;
      c->active = newton;
      return upload_active(c);
    }
    ~Narrowed() { (void)restore(); }
  } nar{c, c->active};
  while (true) {
    e = fetch(c, c->cg(), c->nrve * sizeof(CgState));
    if (e) return e;
    bool all = true;
    int most = 0, running = 0, masked = 0;
    for (int r = 0; r < c->nrve; ++r) {
      const bool done = c->host_cg()[r].done != 0;
      all = all && done;
      most = std::max(most, c->host_cg()[r].iter);
      running += !done;
      masked += c->active[r] != 0;
    }
    if (all) {
      if (most > 0) c->cg_estimate = most;
      if ((e = nar.restore())) return e;
      launch_cg_finish(c->prec, c->launch(), c->x(), c->pw(), c->cg());  // the deferred x updates still due
      return check_launch();
    }
    if (launched > max_cg + 64) return FFTNK_ECG_MAXIT;  // unreachable: k_cg_beta stops at max_cg
    if (running < masked) {
      for (int r = 0; r < c->nrve; ++r) c->active[r] = c->host_cg()[r].done ? 0 : 1;
      nar.on = true;
      if ((e = upload_active(c))) return e;
    }
    e = launch_iterations(c, c->check_every, nar.on);
    if (e) return e;
    launched += c->check_every;
  }
}

int reduce_fetch(fftnk_ctx* c, std::initializer_list<std::pair<int, std::pair<int, int>>> req) {
  const Launch L = c->launch();
  for (const auto& q : req) launch_reduce(L, q.first, q.second.first, q.second.second, c->red());
  const int e = check_launch();
  if (e) return e;
  return fetch(c, c->red(), (size_t)c->nrve * NSLOT * sizeof(double));
}

double red_at(fftnk_ctx* c, int r, int slot) { return c->host_red()[r * NSLOT + slot]; }

// GMRES(m) (Saad, Iterative Methods for Sparse Linear Systems, Alg. 6.9 with
// the Givens update of Sec. 6.5.3) on every active RVE, in the role of run_cg:
// right-hand side b in r (with the partial sums of the right-hand-side
// pipeline), x = 0 on entry, solution in x, per-RVE outcome written to the
// host CgState array that run_cg's callers read (iterations = operator
// applications, the restarts' residual evaluations included).  Arnoldi uses
// classical Gram-Schmidt (one pass over the basis per inner-product batch
// instead of one per vector), repeated where the first pass cancelled more
// than the test of Daniel, Gragg, Kaufman and Stewart allows; the Hessenberg
// columns, rotations and the small triangular solve live on the host.
int run_gmres(fftnk_ctx* c, double eta, int max_it) {
  const int nr = c->nrve, m = c->gm, prec = c->prec;
  const size_t esz = prec == PREC_F64 ? 8 : 4;
  const long long vstride = gm_vstride(c->ntot);
  auto V = [&](int j) { return static_cast<void*>(c->ws + c->o_gm + (size_t)j * vstride * esz); };
  double* coef = c->at<double>(c->o_coef);
  Launch L = c->launch();  // rebuilt whenever the mask changes (launch sizes)
  const Material mat = c->material();
  const std::vector<int> act0 = c->active;  // the caller's mask, restored at the end
  // on an early (error) return the caller's mask is restored all the same
  struct MaskGuard {
    fftnk_ctx* c;
    const std::vector<int>& saved;
    bool armed = true;
    ~MaskGuard() {
      if (!armed) return;
      c->active = saved;
      if (upload_active(c) == FFTNK_OK) (void)hipStreamSynchronize(c->stream);
    }
  } guard{c, act0};
  int e = reduce_fetch(c, {{K_ROW1, {SLOT_YY, 1}}, {K_ROW, {SLOT_BB, 1}}});
  if (e) return e;
  struct RveGm {
    double nb = 0, res = 0;
    int iters = 0, status = FFTNK_OK, done = 0, zero = 0, in_cycle = 0, k = 0;
    std::vector<double> H, cs, sn, g, y, h;
  };
  std::vector<RveGm> R(nr);
  for (int r = 0; r < nr; ++r) {
    RveGm& q = R[r];
    q.H.assign((size_t)(m + 1) * m, 0.0);
    q.cs.assign(m, 0.0);
    q.sn.assign(m, 0.0);
    q.g.assign(m + 1, 0.0);
    q.y.assign(m, 0.0);
    q.h.assign(m + 1, 0.0);
    const double bb = red_at(c, r, SLOT_BB), yy = red_at(c, r, SLOT_YY);
    q.nb = std::sqrt(bb);
    if (!act0[r]) {
      q.done = q.zero = 1;
    } else if (!std::isfinite(bb)) {
      q.done = 1;
      q.status = FFTNK_ENONFINITE;
    } else if (bb == 0.0 || q.nb <= 1e-14 * std::sqrt(yy) || q.nb <= eta * q.nb) {
      q.done = q.zero = 1;
    }
  }
  // host staging of the per-RVE coefficients and the launch mask: both
  // uploads complete before the host vectors are written again
  std::vector<double> hc((size_t)nr * kGmCoef, 0.0);
  auto upload_coef = [&]() -> int {
    HIP_TRY(hipMemcpyAsync(coef, hc.data(), hc.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return FFTNK_OK;
  };
  // sets the launch mask; returns the number of active RVEs, or -status
  auto set_active = [&](auto pred) -> int {
    int any = 0;
    for (int r = 0; r < nr; ++r) {
      c->active[r] = pred(r) ? 1 : 0;
      any += c->active[r];
    }
    const int e2 = upload_active(c);
    if (e2) return -e2;
    L = c->launch();
    return any;
  };
  auto apply_A = [&](const void* v) {  // w = A v
    launch_fwd_a2(prec, FWD_TANGENT, L, mat, v, nullptr, nullptr, nullptr, c->flin(), 1.0, c->spec(), nullptr);
    middle_passes(prec, L, c->spec(), nullptr);
    launch_inv_a2(prec, INV_OUT, L, c->spec(), c->w(), prec, nullptr, 1.0, nullptr);
  };
  bool first = true;
  while (true) {
    // a cycle over every RVE still running; first the residual V_0 = b - A x
    int a = set_active([&](int r) { return !R[r].done && (first || R[r].iters < max_it); });
    if (a < 0) return -a;
    for (int r = 0; r < nr; ++r)
      if (!R[r].done && !c->active[r]) {
        R[r].done = 1;
        R[r].status = FFTNK_ECG_MAXIT;
      }
    if (a == 0) break;
    for (int r = 0; r < nr; ++r) {
      hc[(size_t)r * kGmCoef] = 1.0;
      hc[(size_t)r * kGmCoef + 1] = -1.0;
    }
    if ((e = upload_coef())) return e;
    if (first) {
      launch_gm_lincomb(prec, L, V(0), c->r(), nullptr, coef, true);
    } else {
      apply_A(c->x());
      launch_gm_lincomb(prec, L, V(0), c->r(), c->w(), coef, true);
      for (int r = 0; r < nr; ++r) R[r].iters += c->active[r];
    }
    if ((e = reduce_fetch(c, {{K_ELEM9, {SLOT_RR, 1}}}))) return e;
    for (int r = 0; r < nr; ++r) {
      RveGm& q = R[r];
      q.in_cycle = 0;
      if (!c->active[r]) continue;
      const double beta = std::sqrt(red_at(c, r, SLOT_RR));
      q.res = beta;
      if (!std::isfinite(beta)) {
        q.done = 1;
        q.status = FFTNK_ENONFINITE;
      } else if (beta <= eta * q.nb) {
        q.done = 1;
      } else {
        q.in_cycle = 1;
        q.k = 0;
        std::fill(q.g.begin(), q.g.end(), 0.0);
        q.g[0] = beta;
        hc[(size_t)r * kGmCoef] = 1.0 / beta;
      }
    }
    first = false;
    a = set_active([&](int r) { return R[r].in_cycle != 0; });
    if (a < 0) return -a;
    if (a == 0) continue;
    if ((e = upload_coef())) return e;
    launch_gm_lincomb(prec, L, V(0), V(0), nullptr, coef, false);  // V_0 /= beta
    for (int j = 0; j < m; ++j) {
      a = set_active([&](int r) { return R[r].in_cycle && !R[r].done && R[r].k == j && R[r].iters < max_it; });
      if (a < 0) return -a;
      if (a == 0) break;
      apply_A(V(j));
      for (int r = 0; r < nr; ++r) {
        R[r].iters += c->active[r];
        std::fill(R[r].h.begin(), R[r].h.end(), 0.0);
      }
      // w -= sum_i h_i V_i by classical Gram-Schmidt; a second pass only where
      // the first kept less than 1/sqrt(2) of ||w|| (the "twice is enough"
      // test of Daniel, Gragg, Kaufman and Stewart)
      std::vector<double> w0(nr, 0.0), hn2(nr, 0.0);
      const std::vector<int> act_j = c->active;
      auto take_dots = [&](int i0, int kk) {  // h += d, next coefficients -d
        for (int r = 0; r < nr; ++r)
          for (int q2 = 0; q2 < kk; ++q2) {
            const double d = c->active[r] ? red_at(c, r, SLOT_DOT + q2) : 0.0;
            R[r].h[i0 + q2] += d;
            hc[(size_t)r * kGmCoef + q2] = -d;
          }
      };
      auto need_second = [&](int r) { return c->active[r] && hn2[r] < 0.5 * w0[r]; };
      if (j + 1 <= kGmDot) {
        // one batch: the first pass's update also takes the second pass's
        // inner products, so the basis is read twice, or three times where
        // the second pass is needed
        launch_gm_dots(prec, L, c->w(), V(0), vstride, 0, j + 1, true);
        if ((e = reduce_fetch(c, {{K_ELEM9, {SLOT_DOT, j + 1}}, {K_ELEM9, {SLOT_AUX, 1}}}))) return e;
        for (int r = 0; r < nr; ++r) w0[r] = red_at(c, r, SLOT_AUX);
        take_dots(0, j + 1);
        if ((e = upload_coef())) return e;
        launch_gm_update(prec, L, c->w(), V(0), vstride, 0, j + 1, coef, true, true);
        if ((e = reduce_fetch(c, {{K_ELEM9, {SLOT_DOT, j + 1}}, {K_ELEM9, {SLOT_RR, 1}}}))) return e;
        for (int r = 0; r < nr; ++r)
          if (c->active[r]) hn2[r] = red_at(c, r, SLOT_RR);
        a = set_active(need_second);
        if (a < 0) return -a;
        if (a > 0) {
          take_dots(0, j + 1);
          if ((e = upload_coef())) return e;
          launch_gm_update(prec, L, c->w(), V(0), vstride, 0, j + 1, coef, true);
          if ((e = reduce_fetch(c, {{K_ELEM9, {SLOT_RR, 1}}}))) return e;
          for (int r = 0; r < nr; ++r)
            if (c->active[r]) hn2[r] = red_at(c, r, SLOT_RR);
        }
      } else {
        for (int pass = 0; pass < 2; ++pass) {
          if (pass == 1) {
            a = set_active(need_second);
            if (a < 0) return -a;
            if (a == 0) break;
          }
          for (int i0 = 0; i0 <= j; i0 += kGmDot) {
            const int kk = std::min(kGmDot, j + 1 - i0);
            const bool ww = pass == 0 && i0 == 0;
            launch_gm_dots(prec, L, c->w(), V(0), vstride, i0, kk, ww);
            e = ww ? reduce_fetch(c, {{K_ELEM9, {SLOT_DOT, kk}}, {K_ELEM9, {SLOT_AUX, 1}}})
                   : reduce_fetch(c, {{K_ELEM9, {SLOT_DOT, kk}}});
            if (e) return e;
            if (ww)
              for (int r = 0; r < nr; ++r) w0[r] = red_at(c, r, SLOT_AUX);
            take_dots(i0, kk);
            if ((e = upload_coef())) return e;
            launch_gm_update(prec, L, c->w(), V(0), vstride, i0, kk, coef, i0 + kk == j + 1);
          }
          if ((e = reduce_fetch(c, {{K_ELEM9, {SLOT_RR, 1}}}))) return e;
          for (int r = 0; r < nr; ++r)
            if (c->active[r]) hn2[r] = red_at(c, r, SLOT_RR);
        }
      }
      a = set_active([&](int r) { return act_j[r] != 0; });
      if (a < 0) return -a;
      for (int r = 0; r < nr; ++r) {
        if (!c->active[r]) continue;
        RveGm& q = R[r];
        const double hn = std::sqrt(hn2[r]);
        for (int i = 0; i <= j; ++i) q.H[(size_t)i * m + j] = q.h[i];
        q.H[(size_t)(j + 1) * m + j] = hn;
        hc[(size_t)r * kGmCoef] = hn > 0.0 ? 1.0 / hn : 0.0;
        for (int i = 0; i < j; ++i) {
          const double x0 = q.H[(size_t)i * m + j], x1 = q.H[(size_t)(i + 1) * m + j];
          q.H[(size_t)i * m + j] = q.cs[i] * x0 + q.sn[i] * x1;
          q.H[(size_t)(i + 1) * m + j] = -q.sn[i] * x0 + q.cs[i] * x1;
        }
        const double x0 = q.H[(size_t)j * m + j], x1 = q.H[(size_t)(j + 1) * m + j];
        const double d = std::hypot(x0, x1);
        q.cs[j] = x0 / d;
        q.sn[j] = x1 / d;
        q.H[(size_t)j * m + j] = d;
        q.H[(size_t)(j + 1) * m + j] = 0.0;
        q.g[j + 1] = -q.sn[j] * q.g[j];
        q.g[j] = q.cs[j] * q.g[j];
        q.k = j + 1;
        q.res = std::fabs(q.g[j + 1]);
        if (!std::isfinite(q.res) || !std::isfinite(d) || !(d > 0.0)) {
          q.status = FFTNK_ENONFINITE;
          q.done = 1;
        } else if (q.res <= eta * q.nb || hn == 0.0) {
          q.done = 1;  // converged: x is updated at the end of the cycle
        }
      }
      if ((e = upload_coef())) return e;
      launch_gm_lincomb(prec, L, V(j + 1), c->w(), nullptr, coef, false);  // V_{j+1} = w / h_{j+1,j}
    }
    // x += V y with H y = g (upper triangular, k x k) for every RVE of the cycle
    int kmax = 0;
    for (int r = 0; r < nr; ++r) {
      RveGm& q = R[r];
      if (!q.in_cycle || q.status) continue;
      for (int i = q.k - 1; i >= 0; --i) {
        double t = q.g[i];
        for (int u = i + 1; u < q.k; ++u) t -= q.H[(size_t)i * m + u] * q.y[u];
        q.y[i] = t / q.H[(size_t)i * m + i];
      }
      kmax = std::max(kmax, q.k);
    }
    for (int i0 = 0; i0 < kmax; i0 += kGmCoef) {
      const int kk = std::min(kGmCoef, kmax - i0);
      a = set_active([&](int r) { return R[r].in_cycle && !R[r].status && R[r].k > i0; });
      if (a < 0) return -a;
      for (int r = 0; r < nr; ++r)
        for (int q2 = 0; q2 < kk; ++q2)
          hc[(size_t)r * kGmCoef + q2] = (c->active[r] && i0 + q2 < R[r].k) ? R[r].y[i0 + q2] : 0.0;
      if ((e = upload_coef())) return e;
      launch_gm_update(prec, L, c->x(), V(0), vstride, i0, kk, coef, false);
    }
    e = check_launch();
    if (e) return e;
  }
  // the outcome, where run_cg's callers read it
  CgState* hs = reinterpret_cast<CgState*>(c->pinned);
  for (int r = 0; r < nr; ++r) {
    const RveGm& q = R[r];
    std::memset(&hs[r], 0, sizeof(CgState));
    hs[r].bb = q.nb * q.nb;
    hs[r].rr = q.res * q.res;
    hs[r].iter = q.iters;
    hs[r].done = 1;
    hs[r].status = q.status;
    hs[r].zero_rhs = q.zero;
    hs[r].method = KRYLOV_GMRES;
  }
  guard.armed = false;
  c->active = act0;
  e = upload_active(c);
  if (e) return e;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return check_launch();
}

// Deformation-controlled Newton iterations of Algorithm 1 (Sec. 3.1-3.2) on
// the RVEs with run[r] (the others are left alone: masked off every launch):
// dFbar = Fbar - mean(F_0), first solve with the tangent of F_0, then
// G:K(F_i):dF = -G:P(F_i) until ||dF|| / ||F_0 + dFbar|| < eta_nw and i > 0.
// F_0 is the committed state (warm = false) or the current iterate F (warm =
// true: a further load step from an equilibrium of the same increment).
// Writes F, P (workspace) and, per running RVE, st, status and pbar; commits
// nothing.
int newton_solve(fftnk_ctx* c, const double* Fbar, const std::vector<int>& run, bool warm, double eta_nw,
                 double eta_cg, int max_newton, int max_cg, std::vector<fftnk_stats>& st, std::vector<int>& status,
                 std::vector<double>& pbar) {
  const Range range_("fftnk Newton iterations");
  const int nr = c->nrve;
  std::vector<int> done(nr, 0);
  std::vector<double> Fn(nr, 0.0);
  const Material mat = c->material();
  int e = FFTNK_OK;
  double* F0 = warm ? c->F() : c->Ft();
  for (int r = 0; r < nr; ++r) {
    done[r] = run[r] ? 0 : 1;
    if (!run[r]) continue;
    status[r] = FFTNK_OK;
    for (int k = 0; k < 9; ++k)
      if (!std::isfinite(Fbar[9 * r + k])) {
        status[r] = FFTNK_ENONFINITE;
        done[r] = 1;
      }
  }
  for (int r = 0; r < nr; ++r) c->active[r] = done[r] ? 0 : 1;
  e = upload_active(c);
  if (e) return e;

  // dFbar = Fbar - mean(F_0)  (Sec. 3.1)
  launch_field_sum(c->launch(), F0, SLOT_FBAR);
  e = reduce_fetch(c, {{K_VOX, {SLOT_FBAR, 9}}});
  if (e) return e;
  for (int r = 0; r < nr; ++r)
    for (int k = 0; k < 9; ++k)
      c->uni[9 * r + k] = done[r] ? 0.0 : Fbar[9 * r + k] - red_at(c, r, SLOT_FBAR + k) / (double)c->g[r].n;
  e = upload_uni(c);
  if (e) return e;

  // boundary-condition right-hand side with the tangent of the start state;
  // F = F_0 until the first update adds dFbar
  rhs_pipeline(c, FWD_TANGENT_UNI, nullptr, F0, -1.0);
  launch_set_F(c->launch(), F0, c->F(), c->F32());
  e = reduce_fetch(c, {{K_VOX, {SLOT_FF, 1}}});
  if (e) return e;
  for (int r = 0; r < nr; ++r) Fn[r] = std::sqrt(red_at(c, r, SLOT_FF));

  const double eta_eff = c->prec == PREC_F32 ? std::max(eta_cg, 1e-6) : eta_cg;
  for (int it = 0; it < max_newton; ++it) {
    bool any = false;
    for (int r = 0; r < nr; ++r) any = any || !done[r];
    if (!any) break;
    e = run_cg(c, eta_eff, max_cg);
    if (e) return e;
    for (int r = 0; r < nr; ++r) {
      if (done[r]) continue;
      const CgState& s = c->host_cg()[r];
      st[r].cg_iters[it] = s.iter;
      st[r].cg_relres[it] = (s.bb > 0 && !s.zero_rhs) ? std::sqrt(s.rr / s.bb) : 0.0;
      st[r].n_solves = it + 1;
      if (s.status != FFTNK_OK) {
        status[r] = s.status;
        done[r] = 1;
        c->active[r] = 0;
      }
    }
    e = upload_active(c);
    if (e) return e;
    // F += dF (+ dFbar after the boundary-condition solve), constitutive
    // update; the convergence test; then the new right-hand side -G(P) for
    // the cells still running (its partial sums, which the next CG reads,
    // are laid out by the launch tables of that mask)
    const void* dF = newton_update_source(c);  // FP64 in both precisions
    launch_newton_update(PREC_F64, c->launch(), mat, c->F(), dF, c->P(), c->F32(), it == 0);
    e = reduce_fetch(c, {{K_VOX, {SLOT_DF, 1}}, {K_VOX, {SLOT_PBAR, 9}}, {K_VOX, {SLOT_FAIL, 1}}});
    if (e) return e;
    for (int r = 0; r < nr; ++r) {
      if (done[r]) continue;
      const double res = std::sqrt(red_at(c, r, SLOT_DF)) / Fn[r];
      st[r].newton_res[it] = res;
      bool finite = std::isfinite(res);
      for (int k = 0; k < 9; ++k) {
        pbar[9 * r + k] = red_at(c, r, SLOT_PBAR + k) / (double)c->g[r].n;
        finite = finite && std::isfinite(pbar[9 * r + k]);
      }
      if (red_at(c, r, SLOT_FAIL) > 0.0) {  // the return mapping failed somewhere (e.g. det F <= 0)
        status[r] = FFTNK_EMATERIAL;
        done[r] = 1;
      } else if (!finite) {
        status[r] = FFTNK_ENONFINITE;
        done[r] = 1;
      } else if (res < eta_nw && it > 0) {
        done[r] = 1;  // converged
      } else if (it + 1 >= max_newton) {
        status[r] = FFTNK_ENEWTON_MAXIT;
        done[r] = 1;
      }
      if (done[r]) c->active[r] = 0;
    }
    e = upload_active(c);
    if (e) return e;
    bool more = false;
    for (int r = 0; r < nr; ++r) more = more || !done[r];
    if (more) rhs_pipeline(c, FWD_COPY, c->P(), nullptr, -1.0);
  }
  return FFTNK_OK;
}

// Commit the RVEs with status OK (transactional per RVE: F_t, J2 history),
// copy their F and P out, restore the all-active mask.  *worst: first failure.
int commit_rves(fftnk_ctx* c, const std::vector<int>& status, double* F_dev, double* P_dev, int* worst) {
  const Range range_("fftnk commit");
  *worst = FFTNK_OK;
  for (int r = 0; r < c->nrve; ++r) {
    if (status[r]) {
      if (!*worst) *worst = status[r];
      continue;
    }
    const Grid& g = c->g[r];
    const size_t off = 9 * (size_t)g.vox_off, bytes = 9 * (size_t)g.n * sizeof(double);
    HIP_TRY(hipMemcpyAsync(c->Ft() + off, c->F() + off, bytes, hipMemcpyDeviceToDevice, c->stream));
    if (F_dev) HIP_TRY(hipMemcpyAsync(F_dev + off, c->F() + off, bytes, hipMemcpyDeviceToDevice, c->stream));
    if (P_dev) HIP_TRY(hipMemcpyAsync(P_dev + off, c->P() + off, bytes, hipMemcpyDeviceToDevice, c->stream));
    if (c->model == MODEL_J2)  // store the history of the converged state (Alg. 1)
      for (int k = 0; k < 7; ++k) {
        const size_t o = (size_t)k * c->ntot + g.vox_off;
        HIP_TRY(hipMemcpyAsync(c->at<double>(c->o_hist) + o, c->at<double>(c->o_hnew) + o, g.n * sizeof(double),
                               hipMemcpyDeviceToDevice, c->stream));
      }
  }
  std::fill(c->active.begin(), c->active.end(), 1);
  int e = upload_active(c);
  if (e) return e;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return FFTNK_OK;
}

// Columns m of the macroscopic tangent C[r][i][m] = dPbar_i / dFbar_m at the
// current iterate F (with its FP32 copy) for every (r, m) with want[9 r + m]:
// a unit macroscopic increment E_m spreads as E_m + dF with the boundary-
// condition solve G:K(F):dF = -G:K(F):E_m (Sec. 3.1), so with A w = G(K(F):E_m),
// column m = mean(K(F) : (E_m - w)).  One CG per column index, over all RVEs
// that want it.  Appends one solve per column to st; a failed CG sets status.
int macro_tangent_columns(fftnk_ctx* c, const int* want, double eta_cg, int max_cg, double* C,
                          std::vector<fftnk_stats>& st, std::vector<int>& status) {
  const int nr = c->nrve;
  const double eta_eff = c->prec == PREC_F32 ? std::max(eta_cg, 1e-6) : eta_cg;
  int e = FFTNK_OK;
  for (int m = 0; m < 9; ++m) {
    bool any = false;
    for (int r = 0; r < nr; ++r) {
      c->active[r] = (want[9 * r + m] && !status[r]) ? 1 : 0;
      any = any || c->active[r];
      for (int k = 0; k < 9; ++k) c->uni[9 * r + k] = (c->active[r] && k == m) ? 1.0 : 0.0;
    }
    if (!any) continue;
    e = upload_active(c);
    if (!e) e = upload_uni(c);
    if (e) return e;
    rhs_pipeline(c, FWD_TANGENT_UNI, nullptr, c->F(), +1.0);
    e = run_cg(c, eta_eff, max_cg);
    if (e) return e;
    // the CG outcome, read before the next fetch reuses the host staging buffer
    for (int r = 0; r < nr; ++r) {
      if (!c->active[r]) continue;
      const CgState& s = c->host_cg()[r];
      const int at = st[r].n_solves++;
      if (at < FFTNK_MAX_SOLVES) {
        st[r].cg_iters[at] = s.iter;
        st[r].cg_relres[at] = (s.bb > 0 && !s.zero_rhs) ? std::sqrt(s.rr / s.bb) : 0.0;
      }
      if (s.status != FFTNK_OK) status[r] = s.status;
    }
    const void* w = newton_update_source(c);  // FP64 in both precisions
    launch_tangent_sum(c->launch(), c->material(), c->F(), static_cast<const double*>(w));
    e = reduce_fetch(c, {{K_VOX, {SLOT_PBAR, 9}}});
    if (e) return e;
    for (int r = 0; r < nr; ++r) {
      if (!c->active[r] || status[r]) continue;
      for (int i = 0; i < 9; ++i) C[81 * (size_t)r + 9 * i + m] = red_at(c, r, SLOT_PBAR + i) / (double)c->g[r].n;
    }
  }
  std::fill(c->active.begin(), c->active.end(), 1);
  std::fill(c->uni.begin(), c->uni.end(), 0.0);
  e = upload_active(c);
  if (e) return e;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return FFTNK_OK;
}

// Solve the k x k system A x = r (row-major, stride k) in place in r by
// Gaussian elimination with partial pivoting; false when a pivot falls to
// 1e-12 of the largest entry.
bool solve_small(int k, double* A, double* r) {
  double big = 0.0;
  for (int i = 0; i < k * k; ++i) big = std::fmax(big, std::fabs(A[i]));
  for (int j = 0; j < k; ++j) {
    int piv = j;
    for (int i = j + 1; i < k; ++i)
      if (std::fabs(A[i * k + j]) > std::fabs(A[piv * k + j])) piv = i;
    if (!(std::fabs(A[piv * k + j]) > 1e-12 * big)) return false;
    if (piv != j) {
      for (int q = 0; q < k; ++q) std::swap(A[j * k + q], A[piv * k + q]);
      std::swap(r[j], r[piv]);
    }
    for (int i = j + 1; i < k; ++i) {
      const double f = A[i * k + j] / A[j * k + j];
      for (int q = j; q < k; ++q) A[i * k + q] -= f * A[j * k + q];
      r[i] -= f * r[j];
    }
  }
  for (int j = k - 1; j >= 0; --j) {
    double v = r[j];
    for (int q = j + 1; q < k; ++q) v -= A[j * k + q] * r[q];
    r[j] = v / A[j * k + j];
  }
  return true;
}

}  // namespace

// ===========================================================================
// ---------------------------------------------------------------------------
// plan policies and the autotuner
// ---------------------------------------------------------------------------
int set_plan(fftnk_ctx* c, unsigned pol) {
  if (!policy_valid(pol)) return FFTNK_EINVAL;
  Geo geo;
  const int e = make_geo(c->g, pol, geo);
  if (e) return e;
  if (geo.pstride > c->pstride) return FFTNK_EUNSUPPORTED;
  apply_geo(c, geo);
  c->policy = pol;
  drop_graphs(c);  // the graphs hold the old launch sizes
  if (c->ws) {
    HIP_TRY(hipMemcpyAsync(c->ws + c->o_grids, c->g.data(), c->g.size() * sizeof(Grid), hipMemcpyHostToDevice,
                           c->stream));
    HIP_TRY(hipMemcpyAsync(c->ws + c->o_starts, c->starts.data(), c->starts.size() * sizeof(int),
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));  // the host tables may change again at once
  }
  return FFTNK_OK;
}

// what a policy changes in a context's launches (policies with equal keys
// launch the same kernels on the same tiles)
std::string geo_key(const Geo& geo) {
  std::string k;
  for (const Grid& g : geo.g) {
    const bool lds_col = g.ax[0].reg == 0 || g.ax[1].reg == 0;
    k += std::to_string(g.ax[0].reg) + "," + std::to_string(g.ax[1].reg) + "," + std::to_string(g.ax[2].reg) + "," +
         std::to_string(g.rt) + "," + std::to_string(g.rt1) + "," + std::to_string(lds_col ? g.m64 : 0) + "," +
         std::to_string(lds_col ? g.m32 : 0) + ";";
  }
  return k;
}

// key of the tuning cache: precision, material model, Nyquist choice, cells
std::string tune_key(const fftnk_ctx* c) {
  std::string k = std::to_string(c->prec) + "/" + std::to_string(c->model) + "/" + std::to_string(c->nyq_id);
  for (const Grid& g : c->g)
    k += "/" + std::to_string(g.n0) + "x" + std::to_string(g.n1) + "x" + std::to_string(g.n2);
  return k;
}

std::mutex g_tune_mu;
std::map<std::string, unsigned> g_tuned;  // process-wide: tuning key -> policy

// milliseconds per operator application (x -> w, tangent at the committed
// state F_t), the best of three rounds of `reps` back-to-back applications
int time_operator(fftnk_ctx* c, int reps, const void* flin, double* ms) {
  refresh_j2_tangent(c, flin);
  const Launch L = c->launch();
  const Material mat = c->material();
  auto apply = [&]() {
    launch_fwd_a2(c->prec, FWD_TANGENT, L, mat, c->x(), nullptr, nullptr, nullptr, flin, 1.0, c->spec(), nullptr);
    middle_passes(c->prec, L, c->spec(), nullptr);
    launch_inv_a2(c->prec, INV_OUT, L, c->spec(), c->w(), c->prec, nullptr, 1.0, nullptr);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return FFTNK_EHIP;
  }
  int err = FFTNK_OK;
  double best = 1e300;
  apply();  // first launches of these kernels and tiles
  for (int round = 0; round < 3 && !err; ++round) {
    if (hipEventRecord(e0, c->stream) != hipSuccess) err = FFTNK_EHIP;
    for (int k = 0; k < reps && !err; ++k) apply();
    if (!err && hipEventRecord(e1, c->stream) != hipSuccess) err = FFTNK_EHIP;
    if (!err) err = check_launch();
    if (!err && hipEventSynchronize(e1) != hipSuccess) err = FFTNK_EHIP;
    float t = 0.f;
    if (!err && hipEventElapsedTime(&t, e0, e1) != hipSuccess) err = FFTNK_EHIP;
    if (!err) best = std::min(best, (double)t / reps);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = best;
  return err;
}

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

int fftnk_describe(const fftnk_ctx* c, char* buf, size_t len, size_t* needed) {
  if (!c) return FFTNK_EINVAL;
  std::string j;
  char t[512];
  auto add = [&](const char* fmt, auto... a) {
    std::snprintf(t, sizeof t, fmt, a...);
    j += t;
  };
  add("{\"nrve\": %d, \"precision\": %d, \"workspace_bytes\": %zu, \"workspace_base_bytes\": %zu, \"gmres_restart\": %d, "
      "\"x_window\": %d, \"policy\": %u, \"pstride\": %lld, ",
      c->nrve, c->prec, c->total, c->total_base, c->gm, c->xwin, c->policy, c->pstride);
  j += "\"nblk\": [";
  for (int k = 0; k < NKIND; ++k) add(k ? ", %d" : "%d", c->nblk[k]);
  j += "], \"lds\": [";
  for (int k = 0; k < 8; ++k) add(k ? ", %zu" : "%zu", c->lds[k]);
  add("], \"eng\": [%d, %d, %d], \"cells\": [", c->eng[0], c->eng[1], c->eng[2]);
  for (int r = 0; r < c->nrve; ++r) {
    const Grid& g = c->g[r];
    add("%s{\"n\": [%d, %d, %d], \"h\": %d, \"rows\": %lld, \"vox_off\": %lld, \"spec_off\": %lld, "
        "\"row_off\": %lld, \"rt\": %d, \"rt1\": %d, \"m64\": %d, \"m32\": %d, ",
        r ? ", " : "", g.n0, g.n1, g.n2, g.h, g.rows, g.vox_off, g.spec_off, g.row_off, g.rt, g.rt1, g.m64, g.m32);
    add("\"blocks\": {\"row\": %d, \"row1\": %d, \"col1_64\": %d, \"col1_32\": %d, \"col0_64\": %d, "
        "\"col0_32\": %d, \"elem9\": %d, \"vox\": %d}, \"axes\": [",
        row_blocks(g), row1_blocks(g), col1_blocks(g, PREC_F64), col1_blocks(g, PREC_F32), col0_blocks(g, PREC_F64),
        col0_blocks(g, PREC_F32), elem_blocks(9 * g.n), elem_blocks(g.n));
    for (int d = 0; d < 3; ++d) {
      add("%s{\"n\": %d, \"reg\": %d, \"tw\": %d, \"radix\": [", d ? ", " : "", g.ax[d].n, g.ax[d].reg,
          g.ax[d].tw);
      for (int q = 0; q < g.ax[d].nstages; ++q) add(q ? ", %d" : "%d", g.ax[d].radix[q]);
      j += "]}";
    }
    j += "]}";
  }
  add("], \"tw_total\": %d}", c->tw_total);
  if (needed) *needed = j.size() + 1;
  if (!buf || len < j.size() + 1) return FFTNK_ENOMEM;
  std::memcpy(buf, j.c_str(), j.size() + 1);
  return FFTNK_OK;
}

int fftnk_bind_workspace(fftnk_ctx* c, void* dev, size_t bytes) {
  if (!c || !dev) return FFTNK_EINVAL;
  if ((reinterpret_cast<uintptr_t>(dev) % kAlign) != 0) return FFTNK_EINVAL;
  if (bytes < c->total) return FFTNK_ENOMEM;
  if (!c->pinned && hipHostMalloc(reinterpret_cast<void**>(&c->pinned), c->pinned_bytes) != hipSuccess) {
    c->pinned = nullptr;
    return FFTNK_EHIP;
  }
  if (!c->cap && hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
    c->cap = nullptr;
    return FFTNK_EHIP;
  }
  drop_graphs(c);
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
  HIP_TRY(hipMemcpyAsync(c->ws + c->o_grids, c->g.data(), c->g.size() * sizeof(Grid), hipMemcpyHostToDevice,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(c->ws + c->o_starts, c->starts.data(), c->starts.size() * sizeof(int),
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemsetAsync(c->ws + c->o_cg, 0, (size_t)c->nrve * sizeof(CgState), c->stream));
  HIP_TRY(hipMemsetAsync(c->ws + c->o_part, 0, (size_t)NSLOT * c->pstride * 8, c->stream));
  std::fill(c->active.begin(), c->active.end(), 1);
  std::fill(c->uni.begin(), c->uni.end(), 0.0);
  int e = upload_active(c);
  if (!e) e = upload_uni(c);
  if (e) return e;
  HIP_TRY(hipStreamSynchronize(c->stream));  // the host tables above are temporaries
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
  if (model != FFTNK_SVK && model != FFTNK_J2) return FFTNK_EINVAL;
  if (model == FFTNK_J2 && c->prec != PREC_F64) return FFTNK_EUNSUPPORTED;  // J2 runs in FP64
  if (!c->ws) return FFTNK_ESTATE;
  const int np = model == FFTNK_SVK ? 2 : 4;
  for (int i = 0; i < nphase * np; ++i)
    if (!std::isfinite(params[i])) return FFTNK_EINVAL;
  std::memset(c->mtab, 0, sizeof(c->mtab));
  for (int ph = 0; ph < nphase; ++ph)
    for (int k = 0; k < np; ++k) c->mtab[4 * ph + k] = params[np * ph + k];
  drop_graphs(c);  // captured launches carry the material
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
    if (c->use_mu) drop_graphs(c);  // captured launches carry the material
    c->use_mu = false;
    return FFTNK_OK;
  }
  HIP_TRY(hipMemcpyAsync(c->ws + c->o_mu, mu_dev, (size_t)c->ntot * 8, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (!c->use_mu) drop_graphs(c);
  c->use_mu = true;
  return FFTNK_OK;
}

int fftnk_set_option(fftnk_ctx* c, int option, int value) {
  if (!c) return FFTNK_EINVAL;
  switch (option) {
    case FFTNK_OPT_GRAPHS: c->use_graphs = value != 0; return FFTNK_OK;
    case FFTNK_OPT_CHECK_EVERY:
      if (value < 1 || value > 64) return FFTNK_EINVAL;
      c->check_every = value;
      return FFTNK_OK;
    case FFTNK_OPT_GMRES_RESTART: {
      if (value < 1 || value > 256) return FFTNK_EINVAL;
      if (c->ws) return FFTNK_ESTATE;  // sizes the workspace: set before binding it
      c->gm = value;
      size_workspace(c);
      return FFTNK_OK;
    }
    case FFTNK_OPT_J2_TANGENT:
      if (value != 0 && value != 1) return FFTNK_EINVAL;
      if (c->ws) return FFTNK_ESTATE;  // sizes the workspace: set before binding it
      c->jt = value;
      size_workspace(c);
      return FFTNK_OK;
    case FFTNK_OPT_X_WINDOW:
      if (value < 1 || value > kMaxXWin) return FFTNK_EINVAL;
      if (c->ws) return FFTNK_ESTATE;  // sizes the workspace: set before binding it
      c->xwin = value;
      size_workspace(c);
      return FFTNK_OK;
    case FFTNK_OPT_NYQUIST:
      if (value != 0 && value != 1) return FFTNK_EINVAL;
      if (value == c->nyq_id) return FFTNK_OK;
      c->nyq_id = value;
      for (Grid& g : c->g) g.nyq_id = value;
      drop_graphs(c);  // the graphs hold the pass-3 variant
      if (c->ws) {
        HIP_TRY(hipMemcpyAsync(c->ws + c->o_grids, c->g.data(), c->g.size() * sizeof(Grid), hipMemcpyHostToDevice,
                               c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
      }
      return FFTNK_OK;
    default: return FFTNK_EINVAL;
  }
}

int fftnk_set_plan(fftnk_ctx* c, unsigned policy) {
  if (!c) return FFTNK_EINVAL;
  return set_plan(c, policy);
}

int fftnk_autotune(fftnk_ctx* c, int reps, int use_cache, unsigned* policy, double* ms) {
  const Range range_("fftnk_autotune");
  if (!c || reps < 1 || reps > 1000) return FFTNK_EINVAL;
  if (!c->ws || !c->have_phase || !c->have_mat) return FFTNK_ESTATE;
  const std::string key = tune_key(c);
  if (use_cache) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) {
      const int e = set_plan(c, it->second);
      if (policy) *policy = c->policy;
      if (ms) *ms = -1.0;
      return e;
    }
  }
  const unsigned pol0 = c->policy;
  // inputs: x = 0, the tangent at F_t (FP32 contexts: its FP32 copy in p)
  const size_t esz = c->prec == PREC_F64 ? 8 : 4;
  HIP_TRY(hipMemsetAsync(c->x(), 0, 9 * (size_t)c->ntot * esz, c->stream));
  const void* flin = c->Ft();
  if (c->prec == PREC_F32) {
    launch_convert(PREC_F32, c->Ft(), c->p(), 9 * c->ntot, c->stream);
    flin = c->p();
  }
  std::vector<std::string> seen;
  unsigned best = pol0;
  double best_ms = 1e300;
  for (unsigned pol = 0; pol < kPolicyCodes; ++pol) {
    if (!policy_valid(pol)) continue;
    Geo t;
    if (make_geo(c->g, pol, t) != FFTNK_OK || t.pstride > c->pstride) continue;
    const std::string k = geo_key(t);
    if (std::find(seen.begin(), seen.end(), k) != seen.end()) continue;
    seen.push_back(k);
    double m = 0.0;
    int e = set_plan(c, pol);
    if (!e) e = time_operator(c, reps, flin, &m);
    if (e) {
      (void)set_plan(c, pol0);
      return e;
    }
    if (m < best_ms) {
      best_ms = m;
      best = pol;
    }
  }
  const int e = set_plan(c, best);
  if (e) return e;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[key] = best;
  }
  if (policy) *policy = best;
  if (ms) *ms = best_ms;
  return FFTNK_OK;
}

int fftnk_set_krylov(fftnk_ctx* c, int method, double lo, double hi) {
  if (!c) return FFTNK_EINVAL;
  switch (method) {
    case FFTNK_KRYLOV_CG: break;
    case FFTNK_KRYLOV_CHEBYSHEV:
      if (!(lo > 0.0) || !(hi > lo) || !std::isfinite(hi)) return FFTNK_EINVAL;
      break;
    case FFTNK_KRYLOV_RICHARDSON:
      if (!(lo > 0.0) || !(hi >= lo) || !std::isfinite(hi)) return FFTNK_EINVAL;
      break;
    case FFTNK_KRYLOV_GMRES:
      if (c->gm < 1) return FFTNK_ESTATE;  // no basis in the workspace
      break;
    default: return FFTNK_EINVAL;
  }
  c->krylov = method;
  c->k_lo = lo;
  c->k_hi = hi;
  return FFTNK_OK;
}

int fftnk_reset_state(fftnk_ctx* c) {
  if (!c) return FFTNK_EINVAL;
  if (!c->ws) return FFTNK_ESTATE;
  return reset_state(c);
}

int fftnk_solve_increment(fftnk_ctx* c, const double* Fbar, double eta_nw, double eta_cg, int max_newton, int max_cg,
                          double* F_dev, double* P_dev, double* Pbar, fftnk_stats* stats) {
  const Range range_("fftnk_solve_increment");
  if (!c || !Fbar || !Pbar) return FFTNK_EINVAL;
  if (!(eta_nw > 0) || !(eta_cg > 0) || max_newton < 2 || max_newton > FFTNK_MAX_SOLVES || max_cg < 1)
    return FFTNK_EINVAL;
  if (!c->ws || !c->have_phase || !c->have_mat) return FFTNK_ESTATE;
  const auto t0 = std::chrono::steady_clock::now();
  const int nr = c->nrve;
  std::vector<fftnk_stats> st(nr);
  std::memset(st.data(), 0, nr * sizeof(fftnk_stats));
  std::vector<int> status(nr, FFTNK_OK), run(nr, 1);
  std::vector<double> pbar(9 * (size_t)nr, 0.0);
  int e = newton_solve(c, Fbar, run, false, eta_nw, eta_cg, max_newton, max_cg, st, status, pbar);
  if (e) return e;
  int worst = FFTNK_OK;
  e = commit_rves(c, status, F_dev, P_dev, &worst);
  if (e) return e;
  for (int r = 0; r < nr; ++r)
    if (!status[r])
      for (int k = 0; k < 9; ++k) Pbar[9 * r + k] = pbar[9 * r + k];
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats)
    for (int r = 0; r < nr; ++r) {
      st[r].status = status[r];
      stats[r] = st[r];
      stats[r].t_ms = ms;
    }
  return worst;
}

int fftnk_solve_increment_mixed(fftnk_ctx* c, double* Fbar, const int* mask, const double* Ptarget,
                                double tol_stress, int max_outer, double eta_nw, double eta_cg, int max_newton,
                                int max_cg, double* F_dev, double* P_dev, double* Pbar, fftnk_stats* stats,
                                int* outer) {
  const Range range_("fftnk_solve_increment_mixed");
  if (!c || !Fbar || !mask || !Ptarget || !Pbar) return FFTNK_EINVAL;
  if (!(tol_stress > 0) || max_outer < 1 || !(eta_nw > 0) || !(eta_cg > 0) || max_newton < 2 ||
      max_newton > FFTNK_MAX_SOLVES || max_cg < 1)
    return FFTNK_EINVAL;
  if (!c->ws || !c->have_phase || !c->have_mat) return FFTNK_ESTATE;
  const auto t0 = std::chrono::steady_clock::now();
  const int nr = c->nrve;
  std::vector<fftnk_stats> st(nr), all(nr);
  std::memset(all.data(), 0, nr * sizeof(fftnk_stats));
  std::vector<int> status(nr, FFTNK_OK), run(nr, 1), nout(nr, 0);
  std::vector<double> fb(Fbar, Fbar + 9 * (size_t)nr), pbar(9 * (size_t)nr, 0.0), C(81 * (size_t)nr, 0.0);
  for (int r = 0; r < nr; ++r)
    for (int k = 0; k < 9; ++k)
      if (mask[9 * r + k] && !std::isfinite(Ptarget[9 * r + k])) {
        status[r] = FFTNK_ENONFINITE;
        run[r] = 0;
      }
  auto append = [&](int r, const fftnk_stats& s) {
    for (int j = 0; j < s.n_solves; ++j) {
      const int at = all[r].n_solves++;
      if (at >= FFTNK_MAX_SOLVES) continue;
      all[r].cg_iters[at] = s.cg_iters[j];
      all[r].cg_relres[at] = s.cg_relres[j];
      all[r].newton_res[at] = s.newton_res[j];
    }
  };
  for (int it = 0; it < max_outer; ++it) {
    bool any = false;
    for (int r = 0; r < nr; ++r) any = any || run[r];
    if (!any) break;
    std::memset(st.data(), 0, nr * sizeof(fftnk_stats));
    // deformation-controlled increment at the current Fbar, warm-started from
    // the previous iterate's equilibrium after the first pass
    int e = newton_solve(c, fb.data(), run, it > 0, eta_nw, eta_cg, max_newton, max_cg, st, status, pbar);
    if (e) return e;
    std::vector<int> need(nr, 0);
    for (int r = 0; r < nr; ++r) {
      if (!run[r]) continue;
      append(r, st[r]);
      nout[r] = it + 1;
      if (status[r]) {
        run[r] = 0;
        continue;
      }
      double worst = 0.0;
      for (int k = 0; k < 9; ++k)
        if (mask[9 * r + k]) worst = std::fmax(worst, std::fabs(pbar[9 * r + k] - Ptarget[9 * r + k]));
      if (worst <= tol_stress) {
        run[r] = 0;  // converged
      } else if (it + 1 == max_outer) {
        status[r] = FFTNK_ENEWTON_MAXIT;
        run[r] = 0;
      } else {
        need[r] = 1;
      }
    }
    // masked block of the macroscopic tangent at each unconverged equilibrium,
    // then the outer Newton step on the masked entries of Fbar
    std::vector<int> want(9 * (size_t)nr, 0);
    for (int r = 0; r < nr; ++r)
      for (int k = 0; k < 9; ++k) want[9 * r + k] = need[r] && mask[9 * r + k];
    std::memset(st.data(), 0, nr * sizeof(fftnk_stats));
    // the block only steers the outer step: columns to max(eta_cg, 1e-4)
    e = macro_tangent_columns(c, want.data(), std::max(eta_cg, 1e-4), max_cg, C.data(), st, status);
    if (e) return e;
    for (int r = 0; r < nr; ++r) {
      if (!need[r]) continue;
      append(r, st[r]);
      if (status[r]) {
        run[r] = 0;
        continue;
      }
      int idx[9], k = 0;
      for (int m = 0; m < 9; ++m)
        if (mask[9 * r + m]) idx[k++] = m;
      double A[81], R[9];
      for (int a2 = 0; a2 < k; ++a2) {
        R[a2] = pbar[9 * r + idx[a2]] - Ptarget[9 * r + idx[a2]];
        for (int b2 = 0; b2 < k; ++b2) A[a2 * k + b2] = C[81 * (size_t)r + 9 * idx[a2] + idx[b2]];
      }
      if (!solve_small(k, A, R)) {
        status[r] = FFTNK_EINVAL;  // the mask leaves a direction of Fbar without stress response
        run[r] = 0;
        continue;
      }
      for (int j = 0; j < k; ++j) fb[9 * r + idx[j]] -= R[j];
    }
  }
  int worst = FFTNK_OK;
  int e = commit_rves(c, status, F_dev, P_dev, &worst);
  if (e) return e;
  for (int r = 0; r < nr; ++r) {
    if (outer) outer[r] = nout[r];
    if (status[r]) continue;
    for (int k = 0; k < 9; ++k) {
      Pbar[9 * r + k] = pbar[9 * r + k];
      Fbar[9 * r + k] = fb[9 * r + k];
    }
  }
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats)
    for (int r = 0; r < nr; ++r) {
      all[r].status = status[r];
      all[r].t_ms = ms;
      stats[r] = all[r];
    }
  return worst;
}

int fftnk_macro_tangent(fftnk_ctx* c, const int* want, double eta_cg, int max_cg, double* C_host,
                        fftnk_stats* stats) {
  const Range range_("fftnk_macro_tangent");
  if (!c || !C_host || !(eta_cg > 0) || max_cg < 1) return FFTNK_EINVAL;
  if (!c->ws || !c->have_phase || !c->have_mat) return FFTNK_ESTATE;
  const int nr = c->nrve;
  std::vector<int> w(9 * (size_t)nr, 1), status(nr, FFTNK_OK);
  if (want)
    for (int k = 0; k < 9 * nr; ++k) w[k] = want[k] != 0;
  // linearisation point: the committed state
  const size_t bytes = 9 * (size_t)c->ntot * sizeof(double);
  HIP_TRY(hipMemcpyAsync(c->F(), c->Ft(), bytes, hipMemcpyDeviceToDevice, c->stream));
  if (c->prec == PREC_F32) launch_convert(PREC_F32, c->Ft(), c->F32(), 9 * c->ntot, c->stream);
  std::vector<fftnk_stats> st(nr);
  std::memset(st.data(), 0, nr * sizeof(fftnk_stats));
  std::vector<double> C(81 * (size_t)nr, 0.0);
  int e = macro_tangent_columns(c, w.data(), eta_cg, max_cg, C.data(), st, status);
  if (e) return e;
  int worst = FFTNK_OK;
  for (int r = 0; r < nr; ++r) {
    st[r].status = status[r];
    if (stats) stats[r] = st[r];
    if (status[r] && !worst) worst = status[r];
    for (int k = 0; k < 81; ++k) C_host[81 * (size_t)r + k] = w[9 * r + k % 9] ? C[81 * (size_t)r + k] : 0.0;
  }
  return worst;
}

int fftnk_adjoint(fftnk_ctx* c, const double* gbar, double eta_cg, int max_cg, double* dLdmu, double* dLdK,
                  fftnk_stats* stats) {
  const Range range_("fftnk_adjoint");
  if (!c || !gbar || !dLdmu || !(eta_cg > 0) || max_cg < 1) return FFTNK_EINVAL;
  if (!c->ws || !c->have_phase || !c->have_mat) return FFTNK_ESTATE;
  if (c->model != MODEL_SVK) return FFTNK_EUNSUPPORTED;  // the gradient formula is St. Venant-Kirchhoff's
  const int nr = c->nrve;
  for (int k = 0; k < 9 * nr; ++k)
    if (!std::isfinite(gbar[k])) return FFTNK_ENONFINITE;
  for (int k = 0; k < 9 * nr; ++k) c->uni[k] = gbar[k];
  int e = upload_uni(c);
  if (e) return e;
  // linearisation point: the committed state
  const size_t bytes = 9 * (size_t)c->ntot * sizeof(double);
  HIP_TRY(hipMemcpyAsync(c->F(), c->Ft(), bytes, hipMemcpyDeviceToDevice, c->stream));
  if (c->prec == PREC_F32) launch_convert(PREC_F32, c->Ft(), c->F32(), 9 * c->ntot, c->stream);
  // b = +G(K(F_t) : g), the adjoint of the boundary-condition system
  rhs_pipeline(c, FWD_TANGENT_UNI, nullptr, c->Ft(), +1.0);
  const double eta_eff = c->prec == PREC_F32 ? std::max(eta_cg, 1e-6) : eta_cg;
  e = run_cg(c, eta_eff, max_cg);
  if (e) return e;
  int worst = FFTNK_OK;
  for (int r = 0; r < nr; ++r) {
    const CgState& s = c->host_cg()[r];
    if (stats) {
      std::memset(&stats[r], 0, sizeof(fftnk_stats));
      stats[r].n_solves = 1;
      stats[r].cg_iters[0] = s.iter;
      stats[r].cg_relres[0] = (s.bb > 0 && !s.zero_rhs) ? std::sqrt(s.rr / s.bb) : 0.0;
      stats[r].status = s.status;
    }
    if (s.status && !worst) worst = s.status;
  }
  if (worst) return worst;
  const void* w = newton_update_source(c);
  launch_adjoint_grad(w == c->x() ? c->prec : PREC_F64, c->launch(), c->Ft(), w, dLdmu, dLdK);
  e = check_launch();
  HIP_TRY(hipStreamSynchronize(c->stream));
  return e;
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
  refresh_j2_tangent(c, c->flin());
  const Launch L = c->launch();
  launch_fwd_a2(c->prec, FWD_TANGENT, L, c->material(), p_dev, nullptr, nullptr, nullptr, c->flin(), 1.0, c->spec(),
                nullptr);
  middle_passes(c->prec, L, c->spec(), nullptr);
  launch_inv_a2(c->prec, INV_OUT, L, c->spec(), Ap_dev, c->prec, nullptr, 1.0, nullptr);
  return check_launch();
}

int fftnk_solve_linear(fftnk_ctx* c, const double* b_dev, double* x_dev, double eta, int max_it,
                       fftnk_stats* stats) {
  if (!c || !b_dev || !x_dev || !(eta >= 0) || max_it < 1) return FFTNK_EINVAL;
  if (!c->ws || !c->have_phase || !c->have_mat) return FFTNK_ESTATE;
  // r = G(b) (FP64 projection, rounded to the context precision), x = 0
  rhs_pipeline(c, FWD_COPY, b_dev, nullptr, +1.0);
  const double eta_eff = c->prec == PREC_F32 ? std::max(eta, 1e-6) : eta;
  int e = run_cg(c, eta_eff, max_it);
  if (e) return e;
  int worst = FFTNK_OK;
  for (int r = 0; r < c->nrve; ++r) {
    const CgState& q = c->host_cg()[r];
    if (stats) {
      std::memset(&stats[r], 0, sizeof(fftnk_stats));
      stats[r].n_solves = 1;
      stats[r].cg_iters[0] = q.iter;
      stats[r].cg_relres[0] = (q.bb > 0 && !q.zero_rhs) ? std::sqrt(q.rr / q.bb) : 0.0;
      stats[r].status = q.status;
    }
    if (q.status && !worst) worst = q.status;
  }
  const void* x = newton_update_source(c);  // FP64 in both precisions
  HIP_TRY(hipMemcpyAsync(x_dev, x, 9 * (size_t)c->ntot * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  e = check_launch();
  return e ? e : worst;
}

int fftnk_project(fftnk_ctx* c, const void* a_dev, void* Ga_dev) {
  if (!c || !a_dev || !Ga_dev) return FFTNK_EINVAL;
  if (!c->ws) return FFTNK_ESTATE;
  const Launch L = c->launch();
  launch_fwd_a2(c->prec, FWD_COPY, L, c->material(), a_dev, nullptr, nullptr, nullptr, nullptr, 1.0, c->spec(), nullptr);
  middle_passes(c->prec, L, c->spec(), nullptr);
  launch_inv_a2(c->prec, INV_OUT, L, c->spec(), Ga_dev, c->prec, nullptr, 1.0, nullptr);
  return check_launch();
}

int fftnk_constitutive(fftnk_ctx* c, const double* F_dev, double* P_dev, double* Pbar) {
  if (!c || !F_dev || !P_dev || !Pbar) return FFTNK_EINVAL;
  if (!c->ws || !c->have_phase || !c->have_mat) return FFTNK_ESTATE;
  launch_constitutive(c->launch(), c->material(), F_dev, P_dev);
  const int e = reduce_fetch(c, {{K_VOX, {SLOT_PBAR, 9}}});
  if (e) return e;
  for (int r = 0; r < c->nrve; ++r)
    for (int k = 0; k < 9; ++k) Pbar[9 * r + k] = red_at(c, r, SLOT_PBAR + k) / (double)c->g[r].n;
  return FFTNK_OK;
}

int fftnk_launch_pass(fftnk_ctx* c, int pass) {
  if (!c || pass < 1 || pass > 5) return FFTNK_EINVAL;
  if (!c->ws || !c->have_phase || !c->have_mat) return FFTNK_ESTATE;
  const Launch L = c->launch();
  switch (pass) {
    case 1:
      launch_fwd_a2(c->prec, FWD_TANGENT, L, c->material(), c->p(), nullptr, nullptr, nullptr, c->flin(), 1.0,
                    c->spec(), nullptr);
      break;
    case 2: launch_col_a1(c->prec, false, L, c->spec(), nullptr); break;
    case 3: launch_col_a0_project(c->prec, L, c->spec(), nullptr); break;
    case 4: launch_col_a1(c->prec, true, L, c->spec(), nullptr); break;
    default: launch_inv_a2(c->prec, INV_OUT, L, c->spec(), c->w(), c->prec, nullptr, 1.0, nullptr); break;
  }
  return check_launch();
}

int fftnk_profile_cg(fftnk_ctx* c, int iters, double* ms) {
  if (!c || !ms || iters < 1 || iters > 10000) return FFTNK_EINVAL;
  if (!c->ws || !c->have_phase || !c->have_mat) return FFTNK_ESTATE;
  refresh_j2_tangent(c, c->flin());
  const Launch L = c->launch();
  CgState* cg = c->cg();
  rhs_pipeline(c, FWD_COPY, c->P(), nullptr, -1.0);
  // tolerance 0, no stagnation stop, iteration cap far beyond the launches below
  launch_cg_init(L, cg, 0.0, 1 << 30, 0);
  int e = fetch(c, cg, c->nrve * sizeof(CgState));
  if (e) return e;
  for (int r = 0; r < c->nrve; ++r)
    if (c->host_cg()[r].done) return FFTNK_ESTATE;
  // W + 1 whole iterations untimed (every kernel then sees a previous
  // direction, a window start has passed).  Pass 1, which reads what pass 5
  // of the iteration before wrote, in place: whole iterations with pass 1
  // between two events on the stream, apart at window starts (iteration k
  // with k mod W = 0; every cell runs in step: tolerance 0, no cap).  The
  // other kernels `iters` times back to back between two events (beta last:
  // it advances the iteration counter).
  int err = FFTNK_OK;
  for (int i = 0; i <= c->xwin && !err; ++i) cg_iteration(c, L);
  err = check_launch();
  if (err) return err;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) err = FFTNK_EHIP;
  double s_in = 0, s_start = 0, n_in = 0, n_start = 0;
  const int runs = std::max(iters, c->xwin);
  for (int it = 0, k = c->xwin + 1; it < runs && !err; ++it, ++k) {
    (void)hipEventRecord(e0, c->stream);
    launch_fwd_a2(c->prec, FWD_CG, L, c->material(), nullptr, c->r(), c->pw(), c->x(), c->flin(), 1.0, c->spec(), cg);
    (void)hipEventRecord(e1, c->stream);
    launch_col_a1(c->prec, false, L, c->spec(), cg, cg);  // and alpha
    launch_col_a0_project(c->prec, L, c->spec(), cg);
    launch_col_a1(c->prec, true, L, c->spec(), cg);
    launch_inv_a2(c->prec, INV_CGR, L, c->spec(), c->r(), c->prec, nullptr, 1.0, cg);
    launch_cg_beta(L, cg);
    err = check_launch();
    float t = 0.f;
    if (!err && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess))
      err = FFTNK_EHIP;
    if (err) break;
    if (k % c->xwin == 0) {
      s_start += t;
      n_start += 1;
    } else {
      s_in += t;
      n_in += 1;
    }
  }
  auto kernel = [&](int q) {
    switch (q) {
      case 2: launch_col_a1(c->prec, false, L, c->spec(), cg, cg); break;
      case 3: launch_col_a0_project(c->prec, L, c->spec(), cg); break;
      case 4: launch_col_a1(c->prec, true, L, c->spec(), cg); break;
      case 5: launch_inv_a2(c->prec, INV_CGR, L, c->spec(), c->r(), c->prec, nullptr, 1.0, cg); break;
      default: launch_cg_beta(L, cg); break;
    }
  };
  for (int q = 2; q <= 6 && !err; ++q) {
    (void)hipEventRecord(e0, c->stream);
    for (int i = 0; i < iters; ++i) kernel(q);
    (void)hipEventRecord(e1, c->stream);
    err = check_launch();
    float t = 0.f;
    if (!err && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess))
      err = FFTNK_EHIP;
    ms[q] = (double)t / iters;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (err) return err;
  ms[7] = s_start / std::max(1.0, n_start);
  ms[0] = n_in > 0 ? s_in / n_in : ms[7];  // W = 1: every iteration updates x
  ms[1] = 0.0;                          // alpha: work-groups of pass 2's launch
  return FFTNK_OK;
}

int fftnk_get_history(fftnk_ctx* c, double* hist_dev) {
  if (!c || !hist_dev) return FFTNK_EINVAL;
  if (!c->ws) return FFTNK_ESTATE;
  HIP_TRY(hipMemcpyAsync(hist_dev, c->ws + c->o_hist, 7 * (size_t)c->ntot * 8, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return FFTNK_OK;
}

int fftnk_set_history(fftnk_ctx* c, const double* hist_dev) {
  if (!c || !hist_dev) return FFTNK_EINVAL;
  if (!c->ws) return FFTNK_ESTATE;
  HIP_TRY(hipMemcpyAsync(c->ws + c->o_hist, hist_dev, 7 * (size_t)c->ntot * 8, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
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
  drop_graphs(c);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  if (c->pinned) (void)hipHostFree(c->pinned);
  delete c;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// G projection without a context and without any allocation: the spectrum and
// the launch tables live in one file-scope device array per GPU.  Its host-side
// name is not a device address; the address comes from hipGetSymbolAddress,
// once per device, with that device current.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kNoAllocBytes = (size_t)64 << 20;
constexpr int kNoAllocDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

struct NoAllocDevice {
  char* ptr = nullptr;       // device address of this GPU's copy of `scratch`
  fftnk_ctx* ctx = nullptr;  // host geometry of the cell whose tables the scratch holds
  int key[4] = {0, 0, 0, -1};
};
std::mutex g_noalloc_mu;
NoAllocDevice g_noalloc[kNoAllocDevices];

// compact layout of the projection's buffers inside the scratch; returns the
// bytes needed
size_t noalloc_layout(fftnk_ctx* c) {
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  c->o_grids = take((size_t)c->nrve * sizeof(Grid));
  c->o_starts = take(c->starts.size() * sizeof(int));
  c->o_active = take((size_t)c->nrve * sizeof(int));
  c->o_uni = take((size_t)c->nrve * 9 * sizeof(double));
  c->o_tw64 = take((size_t)c->tw_total * 16);
  c->o_tw32 = take((size_t)c->tw_total * 8);
  c->o_part = take((size_t)NSLOT * c->pstride * 8);
  c->o_spec = take((size_t)c->nspec * (c->prec == PREC_F64 ? 16 : 8));
  // buffers the projection never touches (material, state, Nyquist side
  // buffer: G-hat is zero at Nyquist frequencies here) point at offset 0
  c->o_Ft = c->o_F = c->o_P = c->o_x = c->o_r = c->o_p = c->o_w = c->o_F32 = c->o_d64 = 0;
  c->o_phase = c->o_mu = c->o_hist = c->o_hnew = c->o_mtab = c->o_cg = c->o_red = c->o_nyq = c->o_coef = 0;
  c->o_gm = o;
  c->total = o;
  return o;
}

// tables of a newly planned cell into the scratch (the stream is synchronised:
// the host tables are temporaries)
int noalloc_upload(fftnk_ctx* c) {
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
  const int one = 1;
  HIP_TRY(hipMemcpyAsync(c->ws + c->o_tw64, t64.data(), t64.size() * 8, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->ws + c->o_tw32, t32.data(), t32.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->ws + c->o_grids, c->g.data(), c->g.size() * sizeof(Grid), hipMemcpyHostToDevice,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(c->ws + c->o_starts, c->starts.data(), c->starts.size() * sizeof(int),
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->ws + c->o_active, &one, sizeof(int), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return FFTNK_OK;
}

}  // namespace

extern "C" int fftnk_project_noalloc(int n0, int n1, int n2, int precision, const void* a_dev, void* Ga_dev,
                                     void* hip_stream) {
  if (!a_dev || !Ga_dev) return FFTNK_EINVAL;
  if (precision != FFTNK_FP64 && precision != FFTNK_FP32_MIXED) return FFTNK_EINVAL;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocDevices) return FFTNK_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  NoAllocDevice& d = g_noalloc[dev];
  if (!d.ptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FFTNK_EHIP;
    d.ptr = static_cast<char*>(p);
  }
  const int key[4] = {n0, n1, n2, precision};
  if (!d.ctx || !std::equal(key, key + 4, d.key)) {
    // plan the new cell on the host first: a refused size leaves the
    // scratch's current tables valid
    fftnk_ctx* c = new (std::nothrow) fftnk_ctx();
    if (!c) return FFTNK_EINVAL;
    const int dims[3] = {n0, n1, n2};
    int e = init_ctx(c, 1, dims, precision, hip_stream);
    if (!e && noalloc_layout(c) > kNoAllocBytes) e = FFTNK_ENOMEM;
    if (e) {
      delete c;
      return e;
    }
    c->ws = d.ptr;
    if (d.ctx) delete d.ctx;
    d.ctx = nullptr;
    std::fill(d.key, d.key + 4, 0);
    d.key[3] = -1;
    if ((e = noalloc_upload(c)) != FFTNK_OK) {
      delete c;
      return e;
    }
    d.ctx = c;
    std::copy(key, key + 4, d.key);
  }
  fftnk_ctx* c = d.ctx;
  c->stream = static_cast<hipStream_t>(hip_stream);
  const Launch L = c->launch();
  launch_fwd_a2(c->prec, FWD_COPY, L, c->material(), a_dev, nullptr, nullptr, nullptr, nullptr, 1.0, c->spec(), nullptr);
  middle_passes(c->prec, L, c->spec(), nullptr);
  launch_inv_a2(c->prec, INV_OUT, L, c->spec(), Ga_dev, c->prec, nullptr, 1.0, nullptr);
  return check_launch();
}
