// Internal declarations shared by the kernels and the host driver of libfftnk.
// Not part of the public C-ABI (that is include/fftnk.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace fftnk {

constexpr int kThreads = 256;      // work-group size of every kernel
constexpr int kMaxStages = 12;     // radix stages of one 1-D transform
constexpr int kMaxPhase = 256;     // material phases (every value of the one-byte phase index)
constexpr int kMaxLen = 512;       // longest supported a0 / a1 axis (the LDS engine above kMaxRegLen)
constexpr int kMaxLenA2 = 256;     // longest a2 axis (pass 1 holds a work-group's lines one voxel per thread)
constexpr int kMaxRegLen = 256;    // longest length of the register-resident engine
constexpr int kMaxRve = 256;       // RVEs of one batched context
constexpr int kRedBlocks = 8192;   // most work-groups of an element-wise kernel per RVE
constexpr int kRegP = 8;           // points per thread of the register-resident FFT engine
constexpr int kMaxPpt = 4;         // points per thread of an LDS-engine column tile (n * m <= kMaxPpt * kThreads)
constexpr double kLlcBytes = 256.0 * 1024 * 1024;  // last-level (Infinity) cache of the device
constexpr int kMaxXWin = 8;        // CG directions kept for the windowed update of x (FFTNK_OPT_X_WINDOW)

// LDS padding: entry e of a twiddle table or of a contiguous (unit-stride)
// exchange line sits at e + e / 8, so that eight lanes touching entries 8
// apart (the first Stockham stage writes j * 8 + r) hit distinct banks.
__host__ __device__ constexpr int lpad(int e) { return e + (e >> 3); }
__host__ __device__ constexpr int padded_len(int n) { return n + (n >> 3) + 1; }

// Engine of the a2 forward pass for an a2 plan with `reg` points per thread:
// the 12-point register engine measured slower there than the LDS engine
// (its tangent phase and transform together need more registers), so pass 1
// keeps the LDS engine for those lengths.
__host__ __device__ constexpr int pass1_engine(int reg) { return reg == 12 ? 0 : reg; }

// Radix plan of one 1-D transform of length n: n = prod radix[s].
struct AxisPlan {
  int n;
  int nstages;
  int radix[kMaxStages];
  int tw;   // offset (in complex entries) of the length-n twiddle table W_n^e, e in [0, n)
  int reg;  // points per thread of the register-resident engine: 8 (n = 2^k, 8..256), 12 (n = 3 2^k,
            // 12..192), 0 = LDS engine
};

// One periodic cell (RVE).  Real tensor fields are component-major
// [9][n0][n1][n2]; the cell's block starts at element 9 * vox_off of a field
// buffer.  The half spectrum is [9][n0][n1][h] complex, starting at complex
// element spec_off; h = n2/2 for even n2 (the a2 Nyquist plane, zeroed by the
// projection, is never stored) and (n2+1)/2 for odd n2.
struct Grid {
  int n0, n1, n2, h;
  long long n;      // voxels
  long long rows;   // n0 * n1 grid lines along a2
  long long vox_off;
  long long spec_off;
  long long row_off;  // grid lines of the cells before this one (Nyquist side buffer)
  double inv_n;
  int rt;           // grid lines per work-group in the a2 inverse pass
  int rt1;          // grid lines per work-group in the a2 forward pass (rt1 * n2 <= kThreads)
  int m64, m32;     // pencils per work-group in the LDS-engine a1 / a0 passes (FP64 / FP32)
  int nyq_id;       // G-hat at Nyquist frequencies: 0 zero, 1 identity (App. C)
  AxisPlan ax[3];
};

// FP32 register-engine column passes take their pencils in k2-adjacent pairs
// (one 16-byte access per element for the two) where a work-group's pencils
// would otherwise span fewer than 128 bytes of a spectrum row: register plans
// that leave fewer than 16 pencils per work-group (n = 256), when the half
// line h is even (so that no pair straddles two k2 lines) and the cell's
// spectrum starts on a pair boundary (16-byte aligned).
__host__ __device__ constexpr bool col_pairs32(int pencils_per_group, int h, long long spec_off) {
  return pencils_per_group < 16 && h % 2 == 0 && spec_off % 2 == 0;
}

// Engine of a cell's column pass over an axis (a1 or a0) for elements of esz
// bytes: the axis' register engine (8, 12) or LDS engine (0), or 16 for the
// 8-point register engine on FP32 pencil pairs.
__host__ __device__ constexpr int col_engine(int reg, int n, int h, long long spec_off, int esz) {
  return esz == 4 && reg == 8 && col_pairs32(kThreads / (n / 8), h, spec_off) ? 16 : reg;
}

// Non-temporal streams in single operator applications pay off only where the
// operator's fields (direction, linearisation point, spectrum, result: about
// 36 element sizes per voxel) exceed the last-level cache; on smaller cells
// they cost (96^3: FP32 0.100 -> 0.110 ms, FP64 0.162 -> 0.166 ms).
inline bool op_nontemporal(long long ntot, int esz) { return 36.0 * (double)ntot * esz > kLlcBytes; }

// Launch kinds: every kernel launch covers all RVEs of a context; work-group b
// belongs to RVE r when starts[kind][r] <= b < starts[kind][r + 1].
enum {
  K_ROW = 0,     // a2 inverse pass: grid lines
  K_ROW1,        // a2 forward pass: grid lines
  K_COL1_64,     // a1 pass, FP64
  K_COL1_32,     // a1 pass, FP32
  K_COL0_64,     // a0 + projection pass, FP64
  K_COL0_32,     // a0 + projection pass, FP32
  K_ELEM9,       // element-wise over 9 n values
  K_VOX,         // per voxel
  NKIND
};

// Material: St. Venant-Kirchhoff uses K, mu per phase (lambda = K - 2 mu / 3),
// optionally overridden by a per-voxel shear modulus field.  J2 adds the initial
// yield stress and the linear hardening modulus.
enum { MODEL_SVK = 0, MODEL_J2 = 1 };
struct Material {
  const uint8_t* phase;    // [ntot] phase index per voxel
  const double* mu_field;  // [ntot] per-voxel mu, or null
  const double* table;     // [nphase][4] device table: K, mu, tau_y0, H
  const double* hist;      // J2: committed history [7][ntot] (Cp^-1 xx yy zz xy yz xz, eps_p)
  double* hist_new;        // J2: history of the current iterate [7][ntot]
  const double* j2t;       // J2: compact tangent at the linearisation point [kJ2Tan][ntot], or null (recomputed)
  long long ntot;
  int model;
  int nphase;
};

// Compact J2 tangent per voxel at a linearisation point (frozen history):
// eigenvectors Q of the trial be (9, Q[3 i + a]), the off-diagonal principal
// moduli (3: pairs 01, 12, 02), the diagonal principal block (9, D[3 a + b]),
// the principal Kirchhoff stresses (3).
constexpr int kJ2Tan = 24;

// Slots of block partial sums (FP64); each slot holds one value per work-group
// of the launch that fills it.
enum {
  SLOT_YY = 0,    // ||Y||^2, the field the projection was applied to (RHS)
  SLOT_BB = 1,    // ||b||^2 (RHS)
  SLOT_PW = 2,    // <p, A p>
  SLOT_RR = 3,    // <r, r>
  SLOT_DF = 4,    // ||dF||^2
  SLOT_FF = 5,    // ||F_t + dFbar||^2
  SLOT_PBAR = 6,  // 9 slots: sum of P
  SLOT_FBAR = 15, // 9 slots: sum of F
  SLOT_AUX = 24,  // spare slot (GMRES: ||w||^2)
  SLOT_FAIL = 25, // voxels whose constitutive update failed (Newton update)
  SLOT_DOT = 26,  // kGmDot slots: GMRES inner products <w, v_i>
  NSLOT = 42
};
constexpr int kGmDot = 16;   // basis vectors per GMRES inner-product / update launch
constexpr int kGmCoef = 16;  // per-RVE coefficients of one GMRES update launch
// elements between consecutive GMRES basis vectors: 9 ntot rounded up to an
// even count, so that element pairs start on 2-element boundaries in every
// basis vector
inline long long gm_vstride(long long ntot) { return (9 * ntot + 63) / 64 * 64; }

// Device-resident CG scalars of one RVE.
struct CgState {
  double rr;       // current <r, r>
  double bb;       // <b, b>
  double stop2;    // (eta ||b||)^2
  double alpha, beta, pw;
  double rr_min;   // last recorded minimum of <r, r> (stagnation guard)
  int iter;
  int done;        // 1 once converged or failed: every CG kernel of this RVE is a no-op
  int status;      // 0 running/ok, else an FFTNK_E* code
  int max_cg;
  int stall_limit; // 0: off; else stop when <r, r> has not dropped below 0.75 rr_min for this many iterations
  int since_min;
  int zero_rhs;    // 1: ||b|| at the round-off floor of the projected field, dF = 0
  int x_lo, x_hi;  // the terms alpha_j p_j, x_lo <= j < x_hi, that x still lacks (applied by
                   //    the first pass of an iteration that starts a new window, or by the
                   //    finishing kernel)
  double ahist[kMaxXWin];  // alpha_j at slot j mod W
  int method;      // KRYLOV_*: how alpha and beta are chosen
  double lo, hi;   // spectral bounds of A on range(G) (Chebyshev, Richardson)
  double rho, gam; // Chebyshev recurrence: rho_k and the step gamma_k of the current direction
};

// Krylov methods sharing the fused CG passes (x += alpha p deferred,
// p = r + beta p, r -= alpha A p): CG (alpha, beta from inner products),
// Chebyshev and Richardson (fixed coefficients from [lo, hi]); and GMRES,
// driven from the host over the operator passes and the kernels below.
enum { KRYLOV_CG = 0, KRYLOV_CHEBYSHEV = 1, KRYLOV_RICHARDSON = 2, KRYLOV_GMRES = 3 };
// per-RVE outcome codes of the device Krylov and Newton kernels (CgState::status)
enum { ST_OK = 0, ST_CG_MAXIT = 5, ST_CG_BREAKDOWN = 6, ST_NONFINITE = 8 };

// Everything a launch needs to find its RVE, tables and partial-sum slots.
struct Batch {
  const Grid* grids;    // [nrve] device copy of the grids
  const int* starts;    // [NKIND][nrve + 1] first work-group of each RVE per launch kind
  const int* active;    // [nrve] Newton-level mask: 0 = RVE finished for this increment
  const double* uni;    // [nrve][9] per-RVE uniform tensor (load increment, cotangent, ...)
  const void* tw64;     // double2 twiddle tables
  const void* tw32;     // float2 twiddle tables
  double* partials;     // [NSLOT][pstride]
  long long pstride;
  // identity choice at Nyquist frequencies, even n2: the a2 Nyquist coefficient
  // of every grid line, divided by n2 (pass 1 writes it, pass 5 adds it back;
  // the half spectrum never holds that plane).  Elements of the field type,
  // cell block at 9 row_off, component c of line l at c rows + l.
  void* nyq;
  int nrve;
  // CG directions: W = xwin slots of vstride elements from the p vector, p_j
  // in slot j mod W; x is brought up to date once every W iterations
  int xwin;
  long long vstride;
};

// Modes of the first (a2, forward) pass.
enum {
  FWD_COPY = 0,        // transform the input field itself (scaled)
  FWD_TANGENT = 1,     // transform K(F) : p
  FWD_TANGENT_UNI = 2, // transform K(F) : U with the RVE's uniform tensor U (Batch::uni)
  FWD_CG = 3           // CG iteration k: at the start of a window (k >= W, k mod W = 0)
                       // x += sum of alpha_j p_j over the W previous iterations; then
                       // p_k <- r + beta p_{k-1} (or r when k = 0) in slot k mod W, K(F) : p
                       // and the partial <p, K(F) : p> (= <p, A p>, see cg_alpha_group)
};
// Modes of the last (a2, inverse) pass.
enum {
  INV_OUT = 0,   // write the real field (scaled)
  INV_CGR = 1,   // CG residual: r <- r - alpha w for the transformed field w = A p, partial <r, r>
  INV_RHS = 2    // write r = scale * field (as b), zero x, partial <b, b>
};

enum { PREC_F64 = 0, PREC_F32 = 1 };

// ---- launch geometry (shared by host and kernels) --------------------------
int row_blocks(const Grid& g);
int row1_blocks(const Grid& g);
int col1_blocks(const Grid& g, int prec);
int col0_blocks(const Grid& g, int prec);
int elem_blocks(long long m);

// ---- launchers (fftnk_fft_kernels.hip) ------------------------------------
// nblk_* is the total work-group count of the launch kind (sum over RVEs).
// cg == nullptr: Newton-level launch (RVEs with active == 0 are skipped);
// cg != nullptr: CG launch (RVEs whose CG is done are skipped).
struct Launch {
  Batch b;
  int nblk[NKIND];
  size_t lds_row64, lds_row32, lds_col1_64, lds_col1_32, lds_col0_64, lds_col0_32, lds_row1_64, lds_row1_32;
  int eng[3];  // per grid axis: bit 0 some cell transforms it with the LDS engine, bit 1 / 2 with the 8- / 12-point
               // register engine, bit 3 with the 8-point one on a cell where FP32 takes pencil pairs (col_engine)
  int nyq;     // 1: the cells use the identity choice at Nyquist frequencies (pass 3 variant)
  int ntop;    // 1: single operator applications load the direction and store the result
               //    non-temporally (their fields exceed the last-level cache: op_nontemporal)
  hipStream_t s;
};
void launch_fwd_a2(int prec, int mode, const Launch& L, const Material& mat, const void* in_T, const void* r_T,
                   void* p_T, void* x_T, const void* Flin, double scale, void* spec, const CgState* cg);
// alpha_cg: the launch also computes the CG step lengths (cg_alpha_group) in
// nrve extra work-groups (the forward pass of a CG iteration)
void launch_col_a1(int prec, bool inverse, const Launch& L, void* spec, const CgState* cg, CgState* alpha_cg = nullptr);
void launch_col_a0_project(int prec, const Launch& L, void* spec, const CgState* cg);
void launch_inv_a2(int prec, int mode, const Launch& L, const void* spec, void* out_T, int out_prec, void* x_T,
                   double scale, const CgState* cg);

// ---- launchers (fftnk_solver_kernels.hip) ---------------------------------
void launch_cg_finish(int prec, const Launch& L, void* x_T, const void* p_T, const CgState* cg);
void launch_cg_beta(const Launch& L, CgState* cg);
void launch_cg_init(const Launch& L, CgState* cg, double eta, int max_cg, int stall, int method = KRYLOV_CG,
                    double lo = 0.0, double hi = 0.0);
void launch_set_F(const Launch& L, const double* Ft, double* F, float* Flin32);
void launch_newton_update(int prec, const Launch& L, const Material& mat, double* F, const void* x_T, double* P,
                          float* Flin32, bool add_uni);
void launch_constitutive(const Launch& L, const Material& mat, const double* F, double* P);
// J2: the compact tangent at the linearisation point F into out [kJ2Tan][ntot]
void launch_j2_tangent_data(const Launch& L, const Material& mat, const double* F, double* out);
void launch_field_sum(const Launch& L, const double* X, int slot0);
// out[r * NSLOT + slot0 + s] = sum over RVE r's work-groups of slot slot0 + s, for s < nslots
void launch_reduce(const Launch& L, int kind, int slot0, int nslots, double* out);
void launch_convert(int to_prec, const void* in, void* out, long long count, hipStream_t s);
void launch_set_identity(const Launch& L, double* F);
void launch_set_virgin_history(const Launch& L, double* hist, long long ntot);
void launch_adjoint_grad(int prec, const Launch& L, const double* F, const void* w, double* dmu, double* dK);
// sums of K(F) : (uni - w) per RVE into SLOT_PBAR .. + 8 (w FP64)
void launch_tangent_sum(const Launch& L, const Material& mat, const double* F, const double* w);
// GMRES, element-wise over each active RVE's 9 n values; the basis vector j
// starts at V + j * vstride elements (vstride = gm_vstride(ntot)); coef is a
// device array [nrve][kGmCoef]; k (1..kGmDot) basis vectors V_{i0+q}, q < k,
// per launch.  dots: partial sums of <w, V_{i0+q}> into SLOT_DOT + q, and with
// ww those of ||w||^2 into SLOT_AUX.  update: y += sum_q coef[r][q] V_{i0+q};
// with norm the partial sums of ||y||^2 into SLOT_RR; with dots also those of
// <y, V_{i0+q}> of the updated y into SLOT_DOT + q (and ||y||^2 as with norm).
// lincomb: dst = coef[r][0] s1 + coef[r][1] s2 (s2 may be null, dst may be
// s1); norm as for update.
void launch_gm_dots(int prec, const Launch& L, const void* w, const void* V, long long vstride, int i0, int k,
                    bool ww);
void launch_gm_update(int prec, const Launch& L, void* y, const void* V, long long vstride, int i0, int k,
                      const double* coef, bool norm, bool dots = false);
void launch_gm_lincomb(int prec, const Launch& L, void* dst, const void* s1, const void* s2, const double* coef,
                       bool norm);

}  // namespace fftnk
