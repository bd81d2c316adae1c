// Shared device-side definitions of the pipelined BiCGStab library (gfx950).
//
// Layout conventions
//   * Every solver vector lives in one device arena, padded to a multiple of
//     kPadElems elements with zeros.  The padding stays zero through every
//     recurrence of Algorithm 2 (all inputs of a padded element are zero and
//     operator kernels never write padded rows), so streaming kernels need no
//     bounds checks and can use 16-byte vector loads throughout.
//   * Global reductions (the GLRED phases) are two-level: each block of a
//     streaming kernel writes one FP64 partial per dot product into
//     partials[slot * kMaxPartials + block]; a single "final" block then sums
//     the partials of each slot in a fixed order and updates the device
//     scalar block.  The summation tree is fixed, so results are bitwise
//     reproducible run to run.
//   * All scalar recurrences (alpha, beta, omega, rho) live in FP64 in a
//     device-resident DevScalars block; the host only reads it when polling.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pbcg {

constexpr int kBlock = 256;          // threads per block (4 wave64)
constexpr int kWaves = kBlock / 64;
constexpr int kMaxBlocks = 2048;     // max blocks of an SPMV kernel
constexpr int kMaxPartials = 1024;   // partials per slot = max blocks of a kernel writing partials
constexpr int kNumSlots = 32;        // partial slots
constexpr int64_t kPadElems = 2048;  // vector padding granularity (elements)
constexpr int64_t kWsAlign = 256;    // alignment of every piece of the caller's workspace
constexpr int kXcds = 8;             // MI355X: workgroups are dispatched round-robin over 8 XCDs
constexpr int kSellC = 64;           // SELL slice height = one wavefront
constexpr int kBoundStateArrays = 16;  // arrays of the products reading's per-source state
constexpr int kLdsRows = 1024;       // rows (and threads) of a block of the LDS-window SELL product

// partial slots
enum Slot : int {
  SL_QY = 0,    // (q_i, y_i)                      GLRED 1
  SL_YY = 1,    // (y_i, y_i)
  SL_RR0 = 2,   // (r_0, r_{i+1})                  GLRED 2
  SL_RW0 = 3,   // (r_0, w_{i+1})
  SL_RS0 = 4,   // (r_0, s_i)
  SL_RZ0 = 5,   // (r_0, z_i)
  SL_RR = 6,    // (r_{i+1}, r_{i+1})  (stopping test)
  SL_BB = 7,    // (b, b)              (initialisation)
  // squared norms for the automated replacement bound (Section 3.6)
  SL_K2 = 8, SL_W2 = 9, SL_T2 = 10, SL_M2 = 11, SL_G2 = 12, SL_S2 = 13, SL_L2 = 14,
  SL_Z2 = 15, SL_Q2 = 16, SL_Y2 = 17,          // phase A: k, w, t, m, g, s, l, z, q, y
  SL_X2 = 18, SL_U2 = 19, SL_N2 = 20, SL_V2 = 21,  // phase B: x, u, n, v
  SL_RX2 = 22, SL_RK2 = 23, SL_RL2 = 24,           // replacement: x, k, l after eq:rr
  SL_RS2 = 25, SL_RZ2 = 26,                        // replacement: s, z after eq:rr
};

// final-reduction modes (run by one extra block of an operator kernel, or by
// a one-block kernel)
enum FinalMode : int {
  FIN_NONE = 0,
  FIN_INIT = 1,      // rho_0, alpha_0, ||r_0||, ||b||           (Algorithm 2 initialisation)
  FIN_OMEGA = 2,     // omega_i = (q,y)/(y,y)                    (GLRED 1)
  FIN_BETA = 3,      // beta_{i+1}, alpha_{i+1}, stopping test   (GLRED 2)
  FIN_REDO = 4,      // FIN_BETA after a forced replacement (iteration count unchanged)
  FIN_TRUE = 5,      // ||b - A x|| from slot SL_RR
  FIN_GAP = 6,       // ||(b - A x) - r|| from slot SL_RR into the gap history
  FIN_C_INIT = 7,    // classic: rho_0 = (r0, r0), ||r_0||, ||b||
  FIN_C_ALPHA = 8,   // classic: alpha_i = rho_i / (r0, s_i)
  FIN_C_OMEGA = 9,   // classic: omega_i
  FIN_C_BETA = 10,   // classic: beta_i, stopping test
  FIN_SUM = 11,      // plain sums of slots 0..nslot-1 into DevScalars::sums
  FIN_PROBE = 12,    // the GLRED 2 reduction only (into sig), for kernel timing
};

// done flag values
enum Done : int { RUNNING = 0, RECURSIVE_CONVERGED = 1, STOPPED = 2 };

// status codes (same numbering as the C ABI)
enum Status : int {
  ST_CONVERGED = 0, ST_MAXIT = 1, ST_BREAKDOWN_RHO = 2, ST_BREAKDOWN_OMEGA = 3,
  ST_NONFINITE = 4, ST_TRUE_RES_NOT_MET = 5,
};

// The fields that kernels read in their prologue (the done flag, the flags
// of the replacement decision and the scalars of the vector updates) come
// first, in one 64-byte line: a kernel that tests `done` and then reads the
// scalars finds them in the line the test has already brought in.
struct alignas(64) DevScalars {
  static constexpr bool kProducts = true;   // carries the products reading's state
  int32_t done;                    // Done
  int32_t n_saved;                 // 1: the iteration's pre-replacement z is in the spare vector
  int32_t rr_auto;                 // 1: automated replacement strategy instead of the period
  int32_t rr_next;                 // replacement due in the current iteration (automated)
  int32_t iter;                    // completed iterations
  int32_t rr_period;
  double alpha, beta, omega, omega_prev;
  double rn;
  // (end of the first 64 bytes)
  double tau, rn0, rho, nb, tol;
  int32_t maxit;
  double tr, gap;                  // last true residual norm / last gap norm
  double sig[8];                   // last reduced sums (diagnostics)
  double sums[8];                  // FIN_SUM output
  int32_t status;                  // Status (valid when done == STOPPED)
  int32_t rr_count;                // replacements performed
  int32_t hist_len, gap_len;
  int32_t gap_idx;                 // next free gap-history slot
  int32_t bad_diag;                // set by value-update kernels on a zero diagonal
  // automated residual replacement (running gap bound f^r and eq:criterion)
  int32_t rr_hit;                  // a replacement ran in the current iteration
  int32_t f_ok_prev;               // f^r_i <= tau ||r_i|| at the previous reduction
  int32_t rr_est;                  // 1: square-root estimate instead of the worst-case bound
  int32_t gb_first;                // 1: the next bound step is iteration 0 (initial s, z gaps)
  double eps_b, eps_r;             // epsilon of the recurrences / of a replacement
  double nA, nM, mu, nN;           // ||A||, ||M^-1|| bounds, max nnz per row, N
  double fr, dw, ds_prev, dz_prev; // f^r and the gap-norm bounds
  double pg, ps, pl, pz, pn, pv;   // norms of the iteration i-1 vectors
  double* history;                 // optional ||r_{i+1}|| per iteration
  double* gap_history;             // optional gap norms
  // distributed final reduction: one block per slot stores its sum here, the
  // last block to arrive runs the scalar logic and resets the counter
  double red[kNumSlots];
  int32_t fin_arrive;
  int32_t bound_len;               // entries of bound_history
  double* bound_history;           // optional f^r per iteration (automated mode)
  // the products reading of f^r (moduli of the products of the error
  // propagation matrices): a state per error source in the caller's buffer
  // pr_state, advanced by k_bound_products after each final that moves it
  int32_t gb_prod;                 // 1: products reading (else the nested one above)
  int32_t pr_op;                   // pending work: PR_START | PR_STEP | PR_RESET | PR_CRIT
  int32_t pr_c;                    // current column c (sources 0 .. c+1 in use)
  int32_t pr_first, pr_pending;    // iteration 0 next / B, E, P products await beta
  int32_t pr_its;                  // iteration index for the bound history
  int64_t pr_cap;                  // sources the buffer holds
  double pr_a, pr_b, pr_w, pr_wp;  // signed alpha_i, beta_i, omega_i, omega_{i-1}
  double pr_R, pr_W, pr_S, pr_Z;   // local error group bounds of the step
  double pr_S0, pr_Z0;             // initial s and z gaps (iteration 0)
  double pr_rR, pr_rW, pr_rS, pr_rZ; // gaps of a replacement's recomputation
  double pr_rn;                    // ||r_{i+1}|| for eq:criterion
  double* pr_state;                // 16 arrays of pr_cap doubles
};

// pending work flags of the products reading
enum : int32_t { PR_START = 1, PR_STEP = 2, PR_RESET = 4, PR_CRIT = 8 };

// ----------------------------------------------------------------------------
// reductions
// ----------------------------------------------------------------------------

// The value of lane (lane ^ OFF), for the xor butterfly below: DPP quad
// permutations for 1 and 2 (VALU moves), swizzles within 32 lanes for 4, 8
// and 16 (no address computation), gfx950's permlane32 swap for 32 (after
// the swap of a register with itself, lanes 0-31 find lane + 32 in the
// second result and lanes 32-63 find lane - 32 in the first).
template <int OFF>
__device__ __forceinline__ double lane_xor(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  int plo, phi;
  if constexpr (OFF == 1 || OFF == 2) {
    constexpr int ctrl = OFF == 1 ? 0xB1 : 0x4E;        // quad_perm [1,0,3,2] / [2,3,0,1]
    plo = __builtin_amdgcn_update_dpp(0, lo, ctrl, 0xF, 0xF, false);
    phi = __builtin_amdgcn_update_dpp(0, hi, ctrl, 0xF, 0xF, false);
  } else if constexpr (OFF == 4 || OFF == 8 || OFF == 16) {
    constexpr int pattern = (OFF << 10) | 0x1F;         // bit mode: xor OFF, and 0x1F
    plo = __builtin_amdgcn_ds_swizzle(lo, pattern);
    phi = __builtin_amdgcn_ds_swizzle(hi, pattern);
  } else {
    static_assert(OFF == 32, "butterfly partners are 1, 2, 4, 8, 16, 32");
    const auto slo = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto shi = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    const bool low = (threadIdx.x & 63) < 32;
    plo = (int)(low ? slo[1] : slo[0]);
    phi = (int)(low ? shi[1] : shi[0]);
  }
  return __hiloint2double(phi, plo);
}

// Sum over the 64 lanes of a wavefront as an xor butterfly (partners 32, 16,
// 8, 4, 2, 1): every lane ends with the same bits.
__device__ __forceinline__ double wave_sum(double v) {
  v += lane_xor<32>(v);
  v += lane_xor<16>(v);
  v += lane_xor<8>(v);
  v += lane_xor<4>(v);
  v += lane_xor<2>(v);
  v += lane_xor<1>(v);
  return v;
}

// Wave sums of several values at once, packed four to a register.  gfx950's
// permlane32 swap of two registers leaves, after one add, the pair sums
// (lanes l, l + 32) of one value in the lower half-wave and of the other in
// the upper half; the permlane16 swap of two such results leaves four
// values by 16-lane row (pairs of rows added); DPP rotations within the
// rows (by 8 and 4, then the quad swaps 2 and 1) finish all four rows.  Two
// moves and an add per value pair and step instead of a full butterfly per
// value, and no LDS-pipe swizzle.  Row r of pack p holds value
// 4 p + kRowVal[r]; every value goes through the same adds in the same
// order whatever its place in a pack, and after the row steps all lanes of a
// row hold the same bits (each step adds partners that form the same pair in
// either order).
constexpr int kRowVal[4] = {0, 2, 1, 3};
constexpr int kValLane[4] = {0, 32, 16, 48};   // first lane of the row holding value j

__device__ __forceinline__ double pair_swap32_sum(double a, double b) {
  // lanes 0-31: a_l + a_{l+32}; lanes 32-63: b_{l-32} + b_l
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(a), __double2loint(b), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(a), __double2hiint(b), false,
                                                   false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}

__device__ __forceinline__ double pair_swap16_sum(double a, double b) {
  // rows 0, 2: a_r + a_{r+1}; rows 1, 3: b_{r-1} + b_r
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(a), __double2loint(b), false,
                                                   false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(a), __double2hiint(b), false,
                                                   false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false),
                          __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_f64<0x128>(v);   // row_ror:8
  v += dpp_f64<0x124>(v);   // row_ror:4
  v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
  return v;
}

// the wave sum of each of NS values; store(d, sum) runs in the first lane of
// the row that holds value d
template <int NS, class F>
__device__ __forceinline__ void wave_sums_packed(const double (&v)[NS], F&& store) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int p = 0; p < (NS + 3) / 4; ++p) {
    const int b0 = 4 * p;
    const double a = v[b0];
    const double b = b0 + 1 < NS ? v[b0 + 1 < NS ? b0 + 1 : b0] : 0.0;
    const double P = pair_swap32_sum(a, b);
    double Q = 0.0;
    if (b0 + 2 < NS) {
      const double c = v[b0 + 2 < NS ? b0 + 2 : b0];
      const double d = b0 + 3 < NS ? v[b0 + 3 < NS ? b0 + 3 : b0] : 0.0;
      Q = pair_swap32_sum(c, d);
    }
    const double R = row16_sum(pair_swap16_sum(P, Q));
    const int vi = b0 + kRowVal[lane >> 4];
    if ((lane & 15) == 0 && vi < NS) store(vi, R);
  }
}

// Block-level sum of ND per-thread accumulators; thread d < ND writes the
// block's partial of dot d into partials[slot[d] * kMaxPartials + blk].
template <int ND>
__device__ __forceinline__ void block_partials(double (&acc)[ND], const int (&slot)[ND],
                                               double* __restrict__ partials, int blk) {
  __shared__ double red[ND][kWaves];
  const int wid = threadIdx.x >> 6;
  wave_sums_packed<ND>(acc, [&](int d, double v) { red[d][wid] = v; });
  __syncthreads();
  if (threadIdx.x < ND) {
    const int d = threadIdx.x;
    double s = red[d][0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) s += red[d][w];
    partials[slot[d] * kMaxPartials + blk] = s;
  }
}

// Sums of the first nblk partials of NS slots, computed by one whole block in
// a fixed order (per thread: ascending j; then the wave tree; then the 4 wave
// sums left to right); every thread returns the results.  The loads of up to
// eight slots are issued together before any of them is added: every slot
// holds kMaxPartials entries, so all kMaxPartials / kBlock strides are loaded
// unconditionally (in bounds) and the entries at j >= nblk are not added.
// Guarding each load instead would make each stride wait for the previous
// one, one memory round trip per stride.  The three steps are also available
// separately (slot_loads, slot_thread_sums, block_tree) for kernels that
// issue the loads early and reduce later.
constexpr int kSlotStrides = kMaxPartials / kBlock;

template <int NS>
__device__ __forceinline__ void slot_loads(const double* __restrict__ partials,
                                           const int (&slot)[NS],
                                           double (&p)[NS][kSlotStrides]) {
#pragma unroll
  for (int d = 0; d < NS; ++d) {
#pragma unroll
    for (int u = 0; u < kSlotStrides; ++u)
      p[d][u] = partials[slot[d] * kMaxPartials + u * kBlock + threadIdx.x];
  }
}

template <int NS>
__device__ __forceinline__ void slot_thread_sums(const double (&p)[NS][kSlotStrides], int nblk,
                                                 double (&s)[NS]) {
#pragma unroll
  for (int d = 0; d < NS; ++d) {
    s[d] = 0.0;
#pragma unroll
    for (int u = 0; u < kSlotStrides; ++u)
      if (u * kBlock + (int)threadIdx.x < nblk) s[d] += p[d][u];
  }
}

template <int NS>
__device__ __forceinline__ void block_tree(const double (&s)[NS], double (&out)[NS]) {
  __shared__ double red[NS][kWaves];
  const int wid = threadIdx.x >> 6;
  wave_sums_packed<NS>(s, [&](int d, double v) { red[d][wid] = v; });
  __syncthreads();
#pragma unroll
  for (int d = 0; d < NS; ++d) {
    double t = red[d][0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) t += red[d][w];
    out[d] = t;
  }
  __syncthreads();
}

template <int NS>
__device__ __forceinline__ void block_sum_slots(const double* __restrict__ partials,
                                                const int (&slot)[NS], int nblk,
                                                double (&out)[NS]) {
  constexpr int G = NS < 8 ? NS : 8;
  double s[NS];
#pragma unroll
  for (int d0 = 0; d0 < NS; d0 += G) {
    int sl[G];
    double p[G][kSlotStrides], t[G];
#pragma unroll
    for (int g = 0; g < G; ++g) sl[g] = slot[d0 + g < NS ? d0 + g : d0];
    slot_loads<G>(partials, sl, p);
    slot_thread_sums<G>(p, nblk, t);
#pragma unroll
    for (int g = 0; g < G; ++g)
      if (d0 + g < NS) s[d0 + g] = t[g];
  }
  block_tree<NS>(s, out);
}

// Sum of the first nblk partials of one slot (see block_sum_slots).
__device__ __forceinline__ double block_sum_slot(const double* __restrict__ partials, int slot,
                                                 int nblk) {
  const int sl[1] = {slot};
  double v[1];
  block_sum_slots<1>(partials, sl, nblk, v);
  return v[0];
}

__device__ __forceinline__ bool finite(double v) { return __builtin_isfinite(v); }

// The scalar logic of a final reads and writes a few dozen fields of the
// scalar struct, most of them behind branches, so on global memory every
// access is a dependent round trip.  The block running a final therefore
// copies the struct into LDS with one load per thread, one thread runs the
// logic on the copy, and the block writes the copy back.  While a final
// runs, no other block writes the struct (the other blocks of the kernel
// only read `done`), so writing back every word is safe.
constexpr int kScWords = (int)(sizeof(DevScalars) / 4);
static_assert(sizeof(DevScalars) % 4 == 0, "scalar struct is copied in 32-bit words");
static_assert(kScWords <= 4 * kBlock, "scalar struct copy: at most four words per thread");
static_assert(offsetof(DevScalars, tau) == 64, "prologue fields fill the first 64 bytes");

__device__ __forceinline__ void scalars_to_lds(const DevScalars* __restrict__ sc,
                                               DevScalars* lsc) {
  const uint32_t* src = reinterpret_cast<const uint32_t*>(sc);
  uint32_t* dst = reinterpret_cast<uint32_t*>(lsc);
  for (int i = threadIdx.x; i < kScWords; i += kBlock)
    dst[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
}

__device__ __forceinline__ void scalars_from_lds(DevScalars* __restrict__ sc,
                                                 const DevScalars* lsc) {
  __syncthreads();
  const uint32_t* src = reinterpret_cast<const uint32_t*>(lsc);
  uint32_t* dst = reinterpret_cast<uint32_t*>(sc);
  for (int i = threadIdx.x; i < kScWords; i += kBlock) dst[i] = src[i];
}

// ----------------------------------------------------------------------------
// tile scheduling
// ----------------------------------------------------------------------------

// XCD-aware tile walk.  Block b runs on XCD b % 8; XCD x owns the contiguous
// tile range [x*T/8, (x+1)*T/8) and its blocks stride through it together, so
// tiles that share stencil halo rows are processed by one XCD and hit in its
// L2.  `nwork` must be a multiple of kXcds.
struct XcdWalk {
  int64_t t, end, step;
  __device__ XcdWalk(int64_t ntiles, int blk, int nwork) {
    const int x = blk % kXcds;
    const int j = blk / kXcds;
    const int per = nwork / kXcds;
    const int64_t lo = (ntiles * x) / kXcds;
    end = (ntiles * (x + 1)) / kXcds;
    t = lo + j;
    step = per;
  }
};

// ----------------------------------------------------------------------------
// vector helpers
// ----------------------------------------------------------------------------

typedef double nd2 __attribute__((ext_vector_type(2)));
typedef float nf4 __attribute__((ext_vector_type(4)));
template <typename T> struct V16;                 // 16-byte vector of T
template <> struct V16<double> { typedef nd2 type; static constexpr int n = 2; };
template <> struct V16<float> { typedef nf4 type; static constexpr int n = 4; };

template <typename T>
__device__ __forceinline__ void ld16(const T* __restrict__ p, T (&v)[V16<T>::n]) {
  typedef typename V16<T>::type VT;
  VT t = *reinterpret_cast<const VT*>(p);
  const T* e = reinterpret_cast<const T*>(&t);
#pragma unroll
  for (int k = 0; k < V16<T>::n; ++k) v[k] = e[k];
}

template <typename T>
__device__ __forceinline__ void st16(T* __restrict__ p, const T (&v)[V16<T>::n]) {
  typedef typename V16<T>::type VT;
  VT t;
  T* e = reinterpret_cast<T*>(&t);
#pragma unroll
  for (int k = 0; k < V16<T>::n; ++k) e[k] = v[k];
  *reinterpret_cast<VT*>(p) = t;
}

// Streaming access of C consecutive elements (C a multiple of the 16-byte
// width), optionally with the non-temporal hint (data used once per kernel).
template <typename T, int C, bool NT>
__device__ __forceinline__ void ldc(const T* __restrict__ p, T (&v)[C]) {
  constexpr int W = V16<T>::n;
  typedef typename V16<T>::type VT;
#pragma unroll
  for (int h = 0; h < C / W; ++h) {
    VT t = NT ? __builtin_nontemporal_load(reinterpret_cast<const VT*>(p) + h)
              : reinterpret_cast<const VT*>(p)[h];
    const T* e = reinterpret_cast<const T*>(&t);
#pragma unroll
    for (int k = 0; k < W; ++k) v[h * W + k] = e[k];
  }
}

template <typename T, int C, bool NT>
__device__ __forceinline__ void stc(T* __restrict__ p, const T (&v)[C]) {
  constexpr int W = V16<T>::n;
  typedef typename V16<T>::type VT;
#pragma unroll
  for (int h = 0; h < C / W; ++h) {
    VT t;
    T* e = reinterpret_cast<T*>(&t);
#pragma unroll
    for (int k = 0; k < W; ++k) e[k] = v[h * W + k];
    if (NT) __builtin_nontemporal_store(t, reinterpret_cast<VT*>(p) + h);
    else reinterpret_cast<VT*>(p)[h] = t;
  }
}

// preconditioner kinds (compile-time)
enum PcKind : int { PC_NONE = 0, PC_SCALAR = 1, PC_VECTOR = 2 };

}  // namespace pbcg
