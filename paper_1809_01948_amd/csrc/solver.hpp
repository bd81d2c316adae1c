// Host-side solver state and kernel launchers (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/pbicgstab.h"
#include "common.hpp"
#include "ops.hpp"

namespace pbcg {

// One orientation (A or A^T) of the operator on the device.
struct OpData {
  int kind = OP_SELL;
  // SELL-64
  int64_t nslices = 0;
  int64_t* sptr = nullptr;      // nslices + 1 element offsets
  int32_t* col = nullptr;
  void* val = nullptr;          // T
  int64_t sell_elems = 0;
  int max_width = 0;
  // column window of each block of kLdsRows rows (the columns its rows read
  // and the rows themselves): first column and length, for the product that
  // stages the window in LDS; win_max = the longest window
  int32_t* win_lo = nullptr;
  int32_t* win_len = nullptr;
  int64_t nlb = 0;
  int win_max = 0;
  // stencils
  int dims[3] = {1, 1, 1};
  double c64[7] = {0};
  float c32[7] = {0};
  // DIA5
  void* dia = nullptr;          // T, 5 * ld
};

struct Solver {
  int64_t n = 0, npad = 0, nnz = 0;
  int precision = 0;            // 0 = FP64, 1 = mixed (FP32 storage, FP64 reductions/scalars)
  int precond = 0;              // 0 = none, 1 = Jacobi
  int kind = OP_SELL;
  int pc = PC_NONE;             // compile-time preconditioner kind used by the kernels
  size_t tsize = 8;             // bytes per stored vector element
  OpData A, AT;
  bool have_AT = false;
  // block-Jacobi (block > 0): A holds A M^-1 (M = block diagonal of the
  // input matrix, blocks of `block` rows); Mb = M and Bi = M^-1 as FP64 sliced
  // ELL map the caller's x to the iterate y = M x and back; ytmp is FP64 scratch
  int block = 0;
  OpData Mb, Bi;
  double* ytmp = nullptr;

  // host copies kept for the transpose (built on first use) and value updates
  std::vector<int32_t> h_rowptr, h_col;
  std::vector<double> h_val;
  std::vector<double> h_dia;    // DIA5, 5 * n, S W C E N

  // CSR on the device (gradient on the pattern, value updates)
  int32_t* d_rowptr = nullptr;
  int32_t* d_col = nullptr;
  int64_t* d_posA = nullptr;    // CSR entry -> SELL slot of A
  int64_t* d_posAT = nullptr;   // CSR entry -> SELL slot of A^T
  int64_t* d_diagpos = nullptr; // row -> CSR index of its diagonal (or -1)

  // device memory: pieces of the caller's workspace (ws_used bytes taken)
  char* ws = nullptr;
  size_t ws_size = 0, ws_used = 0;
  std::vector<int64_t> h_pos, h_posAT;   // CSR entry -> SELL slot of A, A^T (host copies)
  void* vec[16] = {nullptr};    // stored solver vectors (T), see VecId
  double* x = nullptr;          // iterate (FP64, padded)
  double* b = nullptr;          // right-hand side (FP64, padded)
  void* dinv = nullptr;         // Jacobi diagonal (T) when a vector is needed
  double dinv_s = 1.0;          // constant Jacobi scale for constant stencils
  double* partials = nullptr;   // kNumSlots * kMaxPartials
  DevScalars* sc = nullptr;       // sc[0] the scalars, sc[1] staging (phase A -> phase B)
  DevScalars* h_sc = nullptr;   // pinned, 2 entries (double-buffered poll)

  int nblk = 8;                 // blocks of every streaming kernel (multiple of 8)
  int nspmv = 8;                // work blocks of the iteration SpMVs (multiple of 8)
  int vnt = 0;                  // non-temporal loads/stores: bit 0 phase A, bit 1 phase B
  bool auto_rr = false;         // the current solve uses the automated replacement
  double normA = 1.0;           // sqrt(||A||_1 ||A||_inf), an upper bound of ||A||_2
  double normM = 1.0;           // max |M^-1|
  int mu_row = 1, mu_col = 1;   // max stored entries per row / per column
  bool spmv_tiled = true;       // several consecutive rows per thread for structured operators
  bool fuse = true;             // phase kernels compute the SPMVs of structured operators
  bool premult = true;          // sliced-ELL products read V_PM (pre_multiplied)
  bool sell_lds = true;         // sliced-ELL iteration products stage their column window in LDS
  int64_t lds_cap = 0;          // bytes of LDS one block may use (device attribute)
  int lds_blocks = 0;           // blocks of the LDS-window product (0: from the window size)
  int small_rpt = 2;            // rows per thread of the single-workgroup solve (1, 2 or 4)
  const double* rhat_in = nullptr;  // the solve's caller shadow vector (null: r_0)
  bool bound_prod = false;      // the solve's gap bound takes the products reading
  bool march3d = true;          // 3D stencil SPMVs march through the grid planes (k_spmv_st3m)
  bool march_phase = true;      // phase kernels visit a 3D grid's tiles plane by plane (TileSeq)
  int march_zlen = 0;           // planes per work item of k_spmv_st3m (0: sized to the grid)
  int64_t vtiles = 0;           // tiles of 256 x (16 bytes / sizeof(T)) elements
  int64_t rtiles = 0;           // tiles of 256 rows

  hipStream_t s1 = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;
  hipEvent_t ev_poll[2] = {nullptr, nullptr};

  // captured iteration chunks: key = (transpose, automated mode, chunk length, start offset
  // mod P, P, gap offset and period, n/v refresh on replacement)
  std::map<std::string, hipGraphExec_t> graphs;
};

enum VecId : int {
  V_RHAT = 0, V_R, V_G, V_S, V_L, V_Z, V_K, V_W, V_T, V_V, V_TMP,
  V_PM,       // M^-1 of the next product's input (sliced ELL with a Jacobi vector)
  V_COUNT
};

// Parameters of a structured operator (stencil or DIA5) for the kernels.
template <typename T>
inline StParams<T> st_params(const Solver& S, const OpData& o) {
  StParams<T> P;
  P.kind = o.kind;
  P.nx = o.dims[0]; P.ny = o.dims[1]; P.nz = o.dims[2];
  for (int d = 0; d < 7; ++d) P.c[d] = sizeof(T) == 8 ? (T)o.c64[d] : (T)o.c32[d];
  P.dia = (const T*)o.dia;
  P.ld = S.npad;
  P.mz = 0;
  return P;
}

// ---- launchers (kernels_vec.hip) ----
// phase A / phase B of Algorithm 2; with a fused operator (fused_kind != 0)
// they also compute t = A M^-1 w and v = A M^-1 z respectively, phase B
// runs the GLRED 1 final in its prologue, and phase A with `pro` the
// previous iteration's GLRED 2 final (fused operators, periodic strategy),
// staging the scalars for the phase B launched with `staged`
// the whole solve in one workgroup (small FP64 systems); false when the
// system or the options do not allow it (nothing launched then); *err
// receives the status of the kernel's LDS-size attribute call
bool launch_small_solve(Solver& S, const pbcg_opts& o, hipStream_t st, hipError_t* err);
void launch_phaseA(Solver& S, bool tr, bool pro, hipStream_t st);
void launch_phaseB(Solver& S, bool tr, bool staged, hipStream_t st);
void launch_final(Solver& S, int mode, int aux, hipStream_t st, bool force = false);
void launch_cl_update(Solver& S, hipStream_t st);
void launch_cl_p(Solver& S, hipStream_t st);
void launch_fill_zero(Solver& S, void* ptr, int64_t count, size_t elem, hipStream_t st);
void launch_to_double(Solver& S, const void* src, double* dst, int64_t n, hipStream_t st);
void launch_set_done(Solver& S, int value, hipStream_t st);
void launch_copy(Solver& S, const double* src, double* dst, hipStream_t st);

// ---- launchers (kernels_op.hip) ----
const OpData& op_of(Solver& S, bool transpose);
// The operator kind whose products the phase kernels compute themselves
// (OP_ST2D5, OP_ST3D7, OP_DIA5), or 0 when the iteration runs separate SPMVs.
int fused_kind(Solver& S, bool transpose);
// Planes per work item when the phase kernels march through a 3D grid
// (TileSeq; 0: row order).  Fused and separate phase kernels use the same
// count, so their dot products are summed in the same order.
int phase_march_planes(Solver& S, bool transpose);
// a GLRED final on its own (one block, or one block per sum beyond eight)
void launch_fin(Solver& S, int fin_mode, hipStream_t st);
void launch_bound_products(Solver& S, hipStream_t st);
void launch_init_res(Solver& S, bool tr, hipStream_t st);
// out = A M^-1 in; with `pre` the input already holds M^-1 applied (V_PM)
void launch_spmv(Solver& S, bool tr, const void* in, void* out, int fin_mode, bool dot_rhat,
                 hipStream_t st, bool pre = false);
// Whether the iteration's two products read V_PM, the copy of their input
// multiplied by the Jacobi vector that phase A, phase B and the replacement
// write beside z and w: sliced ELL with a Jacobi vector, whose product would
// otherwise gather dinv_j beside every z_j (measured: the 2e6 x 27 random
// matrix's product 365 -> ~235 us in FP64).  The products are bitwise those
// of the gathering form (the same multiplication dinv_j * z_j, done once).
bool pre_multiplied(Solver& S, bool transpose);
// the iteration's product on z (V_Z -> V_V) or w (V_W -> V_T)
void launch_iter_spmv(Solver& S, bool tr, int in_vec, int out_vec, int fin_mode, hipStream_t st);
void launch_rr1(Solver& S, bool tr, bool force, hipStream_t st);
void launch_rr2(Solver& S, bool tr, bool force, hipStream_t st, bool save_z = true,
                bool keep_n = true);
// option rr_nv: v = A M^-1 z from the replaced z (predicated like rr1, rr2)
void launch_rr3(Solver& S, bool tr, bool force, hipStream_t st);
void launch_apply_op(Solver& S, const OpData& o, const double* x, double* y, hipStream_t st);
bool sell_lds_ok(const Solver& S, const OpData& o);
void launch_true_res(Solver& S, bool tr, hipStream_t st);
void launch_gap(Solver& S, bool tr, hipStream_t st, bool force = false);
void launch_cl_init(Solver& S, bool tr, hipStream_t st);
void launch_cl_spmv_s(Solver& S, bool tr, hipStream_t st);
void launch_cl_spmv_y(Solver& S, bool tr, hipStream_t st);
void launch_apply(Solver& S, bool tr, const double* x, double* y, hipStream_t st);
void launch_grad(Solver& S, const double* lam, const double* x, double* grad, hipStream_t st);
void launch_update_sell(Solver& S, const double* val_dev, hipStream_t st);
void launch_kappa_assemble(Solver& S, const double* kappa, double cx, double cy, double h,
                           hipStream_t st);
void launch_kappa_grad(Solver& S, const double* lam, const double* x, double* gk, hipStream_t st);


}  // namespace pbcg
