// Internal declarations shared by the kernels and the host driver of libfftnk.
// Not part of the public C-ABI (that is include/fftnk.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace fftnk {

constexpr int kThreads = 256;      // work-group size of every kernel
constexpr int kMaxStages = 12;     // radix stages of one 1-D transform
constexpr int kMaxPhase = 16;      // material phases
constexpr int kMaxLen = 256;       // longest supported grid axis
constexpr int kMaxRve = 256;       // RVEs of one batched context
constexpr int kRedBlocks = 2048;   // grid of the element-wise kernels (partial-sum slots)

// Radix plan of one 1-D transform of length n: n = prod radix[s].
struct AxisPlan {
  int n;
  int nstages;
  int radix[kMaxStages];
  int tw;  // offset (in complex entries) of the length-n twiddle table W_n^e, e in [0, n)
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
  double inv_n;
  int rt;           // grid lines per work-group in the a2 passes
  int m64, m32;     // pencils per work-group in the a1 / a0 passes (FP64 / FP32)
  AxisPlan ax[3];
};

// Material: St. Venant-Kirchhoff uses K, mu per phase (lambda = K - 2 mu / 3),
// optionally overridden by a per-voxel shear modulus field.  J2 adds the initial
// yield stress and the linear hardening modulus.
enum { MODEL_SVK = 0, MODEL_J2 = 1 };
struct Material {
  const uint8_t* phase;    // [n] phase index per voxel
  const double* mu_field;  // [n] per-voxel mu, or null
  const double* table;     // [nphase][4] device table: K, mu, tau_y0, H
  int model;
  int nphase;
};

// Slots of block partial sums (FP64), each kRedBlocks long... the a2 passes may
// use more blocks, so every slot is sized for the largest grid.
enum {
  SLOT_YY = 0,    // ||Y||^2, the field the projection was applied to (RHS)
  SLOT_BB = 1,    // ||b||^2 (RHS)
  SLOT_PW = 2,    // <p, A p>
  SLOT_RR = 3,    // <r, r>
  SLOT_DF = 4,    // ||dF||^2
  SLOT_FF = 5,    // ||F||^2
  SLOT_PBAR = 6,  // 9 slots: sum of P
  SLOT_FBAR = 15, // 9 slots: sum of F
  SLOT_AUX = 24,  // 2 spare slots
  NSLOT = 26
};

// Device-resident CG scalars of one RVE.
struct CgState {
  double rr;       // current <r, r>
  double bb;       // <b, b>
  double stop2;    // (eta ||b||)^2
  double alpha, beta, pw;
  double rr_min;
  int iter;
  int done;        // 1 once converged or failed: every CG kernel of this RVE is a no-op
  int status;      // 0 running/ok, else an FFTNK_E* code
  int max_cg;
  int stall_limit; // 0: off; else stop when rr_min has not improved for this many iterations
  int since_min;
  int pad[2];
};

// Precision-independent launch arguments of one RVE.
struct PassArgs {
  Grid g;
  const void* tw64;  // double2 twiddle tables
  const void* tw32;  // float2 twiddle tables
  double* partials;  // [NSLOT][pstride]
  long long pstride;
  int slot_base;     // per-RVE offset added to partial indices (batched: 0)
};

// Modes of the first (a2, forward) pass.
enum {
  FWD_COPY = 0,        // transform the input field itself (scaled)
  FWD_TANGENT = 1,     // transform K(F) : p
  FWD_TANGENT_UNI = 2, // transform K(F) : U with a uniform U (9 doubles)
  FWD_CG = 3           // p <- r + beta p (or r on the first iteration), then K(F) : p
};
// Modes of the last (a2, inverse) pass.
enum {
  INV_OUT = 0,   // write the real field (scaled)
  INV_PW = 1,    // write w = A p, partial <p, w>
  INV_RHS = 2    // write r = scale * field (as b), zero x, partial <b, b>
};

enum { PREC_F64 = 0, PREC_F32 = 1 };

// ---- launchers (fftnk_kernels.hip) ----------------------------------------
// prec selects the storage / arithmetic type of the transforms and of the
// vectors named "T" below; F, P, material data are always FP64 except Flin32.
void launch_fwd_a2(int prec, int mode, const PassArgs& a, const Material& mat, const void* in_T,
                   const void* r_T, void* p_T, const void* Flin, const double* uni, double scale,
                   void* spec, const CgState* cg, hipStream_t s);
void launch_col_a1(int prec, bool inverse, const PassArgs& a, void* spec, const CgState* cg, hipStream_t s);
void launch_col_a0_project(int prec, const PassArgs& a, void* spec, const CgState* cg, hipStream_t s);
void launch_inv_a2(int prec, int mode, const PassArgs& a, const void* spec, void* out_T, int out_prec,
                   const void* p_T, void* x_T, double scale, const CgState* cg, hipStream_t s);

void launch_cg_update(int prec, const PassArgs& a, void* x_T, void* r_T, const void* p_T, const void* w_T,
                      CgState* cg, hipStream_t s);
void launch_cg_alpha(const PassArgs& a, int nblk_pw, CgState* cg, hipStream_t s);
void launch_cg_beta(const PassArgs& a, CgState* cg, hipStream_t s);
void launch_cg_init(const PassArgs& a, int nblk_bb, CgState* cg, double eta, int max_cg, int stall,
                    hipStream_t s);

void launch_set_F(const PassArgs& a, const double* Ft, double* F, const double* dFbar, float* Flin32,
                  hipStream_t s);
void launch_newton_update(int prec, const PassArgs& a, const Material& mat, double* F, const void* x_T,
                          double* P, float* Flin32, hipStream_t s);
void launch_constitutive(const PassArgs& a, const Material& mat, const double* F, double* P, hipStream_t s);
void launch_field_sum(const PassArgs& a, const double* X, int slot0, hipStream_t s);
void launch_reduce(const PassArgs& a, int slot0, int nslots, int nblk, double* out, hipStream_t s);
void launch_convert(int to_prec, const void* in, void* out, long long count, hipStream_t s);
void launch_fill_zero(int prec, void* x, long long count, hipStream_t s);
void launch_set_identity(const PassArgs& a, double* F, hipStream_t s);
void launch_adjoint_grad(int prec, const PassArgs& a, const double* F, const void* w, const double* g, double* dmu,
                         double* dK, long long out_off, hipStream_t s);

int fwd_a2_blocks(const Grid& g);
int elem_blocks_vox(const Grid& g);
int inv_a2_blocks(const Grid& g);

}  // namespace fftnk
