// Streaming kernels of pipelined BiCGStab: the two fused multi-AXPY passes
// (with their dot-product partials), the classic method's vector updates,
// and the one-block final reduction kernel.
//
// Each thread owns one 16-byte chunk (2 doubles or 4 floats) per tile, so a
// wave moves 1 KiB per vector per tile with fully coalesced dwordx4 accesses.
// Vectors are zero-padded to whole tiles: no bounds checks.

#include <stdexcept>
#include <type_traits>

#include "solver.hpp"

namespace pbcg {

template <typename T>
struct PhaseAArgs {
  const T* __restrict__ k;
  const T* __restrict__ w;
  T* __restrict__ t;                // read, or written when the product is fused
  const T* __restrict__ r;
  const T* __restrict__ v;
  T* __restrict__ g;
  T* __restrict__ s;
  T* __restrict__ l;
  T* __restrict__ z;
  const T* __restrict__ zsave;     // pre-replacement z_{i-1} (when a replacement preceded)
  T* __restrict__ pm;               // n_i = M^-1 z_i for the next product, or null
  const T* __restrict__ dinv;
  T dinv_s;
};

// Phase A: the four auxiliary recurrences of Algorithm 2 for iteration i
//   g_i = k_i + beta_i (g_{i-1} - omega_{i-1} l_{i-1})
//   s_i = w_i + beta_i (s_{i-1} - omega_{i-1} z_{i-1})
//   l_i = m_i + beta_i (l_{i-1} - omega_{i-1} n_{i-1})   m_i = M^-1 w_i, n_{i-1} = M^-1 z_{i-1}
//   z_i = t_i + beta_i (z_{i-1} - omega_{i-1} v_{i-1})
// in place, and the GLRED 1 partials (q_i, y_i), (y_i, y_i) with
// q_i = r_i - alpha_i s_i, y_i = w_i - alpha_i z_i formed in registers.
// In iteration 0 the previous vectors are zero and beta_0 = 0.  After a
// residual replacement (SAVED) n_{i-1} is formed from the saved
// pre-replacement z_{i-1} instead of the replaced one.  NT selects
// non-temporal loads and stores; AUTO adds the squared norms of k, w, t, m,
// g, s, l, z, q, y that the automated replacement bound needs.
//
// KIND != 0 (a structured operator): t_i = A m_i = A M^-1 w_i is computed
// here from w_i, which is final when this kernel starts, instead of being
// read (the SPMV that the unfused iteration runs after GLRED 2), and
// stored.  w is then read with cached loads so that the stencil neighbours
// of other tiles are served by the L2 of the XCD that walks them.
// Registers of one phase A chunk
template <typename T>
struct ATile {
  static constexpr int C = V16<T>::n;
  T k[C], w[C], t[C], r[C], v[C], g[C], s[C], l[C], z[C], zp[C], d[C], m[C];
  T pd[C], pu[C];     // plane march, 3D: w a plane below and above (as stored)
};

// the loads of one chunk
template <typename T, int PC, bool NT, int KIND, bool SAVED>
__device__ __forceinline__ void phaseA_issue(const PhaseAArgs<T>& A, int64_t i, ATile<T>& R,
                                             bool have_w = false) {
  constexpr int C = V16<T>::n;
  constexpr bool FUSE = KIND != 0;
  ldc<T, C, NT>(A.k + i, R.k);
  if (!have_w) ldc<T, C, NT && !FUSE>(A.w + i, R.w);
  if (!FUSE) ldc<T, C, NT>(A.t + i, R.t);
  ldc<T, C, NT>(A.r + i, R.r); ldc<T, C, NT>(A.v + i, R.v); ldc<T, C, NT>(A.g + i, R.g);
  ldc<T, C, NT>(A.s + i, R.s); ldc<T, C, NT>(A.l + i, R.l); ldc<T, C, NT>(A.z + i, R.z);
  if (SAVED) ldc<T, C, NT>(A.zsave + i, R.zp);
  if (PC == PC_VECTOR) ldc<T, C, NT>(A.dinv + i, R.d);
}

// The first tile of a phase A with the GLRED 2 prologue: its eight streams
// k, w, r, v, g, s, l, z are loaded straight into LDS (16-byte global-to-LDS
// loads, no registers held) before the prologue's reduction, so the
// reduction and the tile's loads overlap.  LDS: one 4 KiB slab per stream,
// lane l of wave v at byte 1024 v + 16 l (the order the loads write).
constexpr int kPfArrays = 8;
constexpr int kPfBytes = kPfArrays * kBlock * 16;

typedef __attribute__((address_space(3))) void lds_void;   // an LDS address

template <typename T>
__device__ __forceinline__ void phaseA_prefetch(const PhaseAArgs<T>& A, int64_t i, char* pf) {
  char* wave = pf + (threadIdx.x >> 6) * 1024;
  const T* src[kPfArrays] = {A.k, A.w, A.r, A.v, A.g, A.s, A.l, A.z};
#pragma unroll
  for (int a = 0; a < kPfArrays; ++a)
    __builtin_amdgcn_global_load_lds((const void*)(src[a] + i),
                                     (lds_void*)(wave + a * kBlock * 16), 16, 0, 0);
}

// waits for the prefetch (vmcnt counts it) before the LDS copies are read
__device__ __forceinline__ void prefetch_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// the prefetched streams from LDS, then the loads that were not prefetched
template <typename T, int PC, bool NT, int KIND, bool SAVED>
__device__ __forceinline__ void phaseA_take(const PhaseAArgs<T>& A, int64_t i, const char* pf,
                                            ATile<T>& R) {
  constexpr int C = V16<T>::n;
  typedef typename V16<T>::type VT;
  prefetch_wait();
  const char* me = pf + threadIdx.x * 16;
  T* dst[kPfArrays] = {R.k, R.w, R.r, R.v, R.g, R.s, R.l, R.z};
#pragma unroll
  for (int a = 0; a < kPfArrays; ++a) {
    const VT x = *reinterpret_cast<const VT*>(me + a * kBlock * 16);
#pragma unroll
    for (int e = 0; e < C; ++e) dst[a][e] = x[e];
  }
  if (KIND == 0) ldc<T, C, NT>(A.t + i, R.t);
  if (SAVED) ldc<T, C, NT>(A.zsave + i, R.zp);
  if (PC == PC_VECTOR) ldc<T, C, NT>(A.dinv + i, R.d);
}

// Whether a phase kernel can march (3D products fused, or none fused: the
// separate-product kernels follow the same order); the 2D kernels keep the
// row order compiled in
template <int KIND>
__device__ __forceinline__ constexpr bool marchable() {
  return KIND == OP_ST3D7 || KIND == 0;
}
template <int KIND, typename T>
__device__ __forceinline__ auto tile_seq(int64_t ntiles, int C, const StParams<T>& P) {
  if constexpr (marchable<KIND>()) return TileSeq(ntiles, C, P.nx, P.ny, P.nz, P.mz);
  else return RowSeq(ntiles, C);
}

// Whether a phase kernel computes a 3D product with the planes below and
// above in registers: plane march over a 3D grid, the product fused (a 3D
// stencil's Jacobi scale is a scalar, never a vector)
template <int KIND, int PC, typename T>
__device__ __forceinline__ bool march_fused(const StParams<T>& P) {
  if constexpr (KIND == OP_ST3D7 && PC != PC_VECTOR) return P.mz > 0;
  return false;
}

// m = M^-1 w of one chunk and, fused, t = A m from the neighbours of w
template <typename T, int PC, int KIND, bool NT>
__device__ __forceinline__ void phaseA_stencil(const PhaseAArgs<T>& A, const StParams<T>& P,
                                               int64_t n, int64_t i, ATile<T>& R) {
  constexpr int C = V16<T>::n;
#pragma unroll
  for (int e = 0; e < C; ++e) {
    const T de = (PC == PC_VECTOR) ? R.d[e] : A.dinv_s;
    R.m[e] = (PC == PC_NONE) ? R.w[e] : de * R.w[e];
  }
  if constexpr (KIND != 0) {
    if (march_fused<KIND, PC>(P)) {
      // plane march: the planes below and above come from registers
      T xd[C], xu[C];
#pragma unroll
      for (int e = 0; e < C; ++e) {
        xd[e] = prec1<T, PC>(R.pd[e], nullptr, A.dinv_s, 0);
        xu[e] = prec1<T, PC>(R.pu[e], nullptr, A.dinv_s, 0);
      }
      st_apply3_planes<T, PC>(P, A.w, A.dinv, A.dinv_s, (int)i, xd, R.m, xu, R.t);
    } else if (i < n) {
      st_apply<T, PC, KIND, 1, NT && sizeof(T) == 8>(P, A.w, A.dinv, A.dinv_s, (int)i, R.m,
                                                     R.t);
    } else {
#pragma unroll
      for (int e = 0; e < C; ++e) R.t[e] = T(0);          // padding rows stay zero
    }
  }
}

// Plane march over a 3D grid with the product fused: w of the tile a plane
// below and above.  A tile that continues its item takes its own w and the
// plane below from the previous tile's registers (`have_w`), so each plane
// of w is loaded once per item, plus the plane before it.
template <typename T>
__device__ __forceinline__ void march_rotate(T (&w)[V16<T>::n], T (&pd)[V16<T>::n],
                                             T (&pu)[V16<T>::n]) {
#pragma unroll
  for (int e = 0; e < V16<T>::n; ++e) {
    pd[e] = w[e];
    w[e] = pu[e];
  }
}
template <typename T>
__device__ __forceinline__ void march_planes(const T* __restrict__ w, const TileSeq& it,
                                             T (&pd)[V16<T>::n], T (&pu)[V16<T>::n]) {
  constexpr int C = V16<T>::n;
  if (!it.cont && it.k > 0) ldc<T, C, false>(w + it.row() - it.nxy, pd);
  if (it.k < it.nz - 1) ldc<T, C, false>(w + it.row() + it.nxy, pu);
}

// the recurrences of one chunk and their partials
template <typename T, int PC, bool NT, bool AUTO, int KIND, bool SAVED>
__device__ __forceinline__ void phaseA_update(const PhaseAArgs<T>& A, int64_t i, ATile<T>& R,
                                              T a, T b, T wp, double (&acc)[12]) {
  constexpr int C = V16<T>::n;
  constexpr bool FUSE = KIND != 0;
#pragma unroll
  for (int e = 0; e < C; ++e) {
    const T de = (PC == PC_VECTOR) ? R.d[e] : A.dinv_s;
    const T zprev = SAVED ? R.zp[e] : R.z[e];
    const T np = (PC == PC_NONE) ? zprev : de * zprev;
    const T gn = R.k[e] + b * (R.g[e] - wp * R.l[e]);
    const T sn = R.w[e] + b * (R.s[e] - wp * R.z[e]);
    const T ln = R.m[e] + b * (R.l[e] - wp * np);
    const T zn = R.t[e] + b * (R.z[e] - wp * R.v[e]);
    const T q = R.r[e] - a * sn;
    const T y = R.w[e] - a * zn;
    acc[0] += (double)q * (double)y;
    acc[1] += (double)y * (double)y;
    if (AUTO) {
      acc[2] += (double)R.k[e] * (double)R.k[e];
      acc[3] += (double)R.w[e] * (double)R.w[e];
      acc[4] += (double)R.t[e] * (double)R.t[e];
      acc[5] += (double)R.m[e] * (double)R.m[e];
      acc[6] += (double)gn * (double)gn;
      acc[7] += (double)sn * (double)sn;
      acc[8] += (double)ln * (double)ln;
      acc[9] += (double)zn * (double)zn;
      acc[10] += (double)q * (double)q;
      acc[11] += (double)y * (double)y;
    }
    R.g[e] = gn; R.s[e] = sn; R.l[e] = ln; R.z[e] = zn;
  }
  stc<T, C, NT>(A.g + i, R.g); stc<T, C, NT>(A.s + i, R.s); stc<T, C, NT>(A.l + i, R.l);
  stc<T, C, NT>(A.z + i, R.z);
  if (FUSE) stc<T, C, NT>(A.t + i, R.t);
  if constexpr (!FUSE && PC == PC_VECTOR) {
    if (A.pm) {                       // n_i = M^-1 z_i, the next product's input
      T pn[C];
#pragma unroll
      for (int e = 0; e < C; ++e) pn[e] = R.d[e] * R.z[e];
      stc<T, C, NT>(A.pm + i, pn);
    }
  }
}

// Inputs of the prologue's GLRED 2 step, loaded at kernel entry
struct G2In {
  double omega, rho, tol, nb;
  int done, its, maxit;
  double pp[5][kSlotStrides];           // the GLRED 2 partials of this thread
};

// The prologue GLRED 2 step (see k_phaseA): every thread evaluates it from
// the reduced sums with the same expressions as run_final; block 0 also runs
// run_final on an LDS copy of the struct, with the history log, and stages
// the copy in sc[1].  Returns whether this iteration runs (and its scalars).
__device__ __forceinline__ bool phaseA_prologue(DevScalars* __restrict__ sc, const G2In& in,
                                                double& alpha, double& beta, double& omega_prev) {
  __shared__ DevScalars lsc;
  __shared__ double pre[kNumSlots];
  const int tid = threadIdx.x;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(sc);
  uint32_t w0 = 0, w1 = 0;
  if (blockIdx.x == 0) {
    if (tid < kScWords) w0 = src[tid];
    if (tid + kBlock < kScWords) w1 = src[tid + kBlock];
  }
  const int sl[5] = {SL_RR0, SL_RW0, SL_RS0, SL_RZ0, SL_RR};
  double ts[5], v[5];
  slot_thread_sums<5>(in.pp, gridDim.x, ts);
  if (blockIdx.x == 0) {
    uint32_t* dl = reinterpret_cast<uint32_t*>(&lsc);
    if (tid < kScWords) dl[tid] = w0;
    if (tid + kBlock < kScWords) dl[tid + kBlock] = w1;
  }
  block_tree<5>(ts, v);                   // (its barriers also publish lsc)
  const G2Step g = glred2_step(v, alpha, in.omega, in.rho, in.tol, in.nb);
  if (blockIdx.x == 0) {
    if (tid == 0 && !in.done) {           // (a stopped solve is staged unchanged)
#pragma unroll
      for (int d = 0; d < 5; ++d) pre[sl[d]] = v[d];
      run_final(FIN_BETA, &lsc, pre, 0);
    }
    scalars_from_lds(sc + 1, &lsc);
  }
  // (with its == maxit the step is taken and the solve then stops, as in
  // run_final, with no iteration left to run)
  if (in.done || g.outcome != G2_CONTINUE || in.its >= in.maxit) return false;
  beta = g.beta;
  alpha = g.alpha;
  omega_prev = in.omega;
  return true;
}

// Phase A over the block's chunks
template <typename T, int PC, bool NT, bool AUTO, int KIND, bool SAVED, bool PF>
__device__ __forceinline__ void phaseA_body(const PhaseAArgs<T>& A, const StParams<T>& P, int64_t n,
                                            double* __restrict__ partials, int64_t ntiles,
                                            double alpha, double beta, double omega_prev,
                                            const char* pf) {
  constexpr int C = V16<T>::n;
  auto it = tile_seq<KIND>(ntiles, C, P);
  const bool mw = march_fused<KIND, PC>(P);      // fused 3D product, planes in registers
  ATile<T> R;
  if (it.valid() && it.has) {
    if constexpr (PF) phaseA_take<T, PC, NT, KIND, SAVED>(A, it.row(), pf, R);
    else phaseA_issue<T, PC, NT, KIND, SAVED>(A, it.row(), R);
    if constexpr (marchable<KIND>()) if (mw) march_planes<T>(A.w, it, R.pd, R.pu);
    phaseA_stencil<T, PC, KIND, NT>(A, P, n, it.row(), R);
  }
  const T a = (T)alpha, b = (T)beta, wp = (T)omega_prev;
  double acc[12];
#pragma unroll
  for (int d = 0; d < 12; ++d) acc[d] = 0.0;
  while (it.valid()) {
    if (it.has) phaseA_update<T, PC, NT, AUTO, KIND, SAVED>(A, it.row(), R, a, b, wp, acc);
    it.next();
    if (it.valid() && it.has) {
      const bool carry = mw && it.cont;
      if (carry) march_rotate<T>(R.w, R.pd, R.pu);
      phaseA_issue<T, PC, NT, KIND, SAVED>(A, it.row(), R, carry);
      if constexpr (marchable<KIND>()) if (mw) march_planes<T>(A.w, it, R.pd, R.pu);
      phaseA_stencil<T, PC, KIND, NT>(A, P, n, it.row(), R);
    }
  }
  if (AUTO) {
    const int slots[12] = {SL_QY, SL_YY, SL_K2, SL_W2, SL_T2, SL_M2, SL_G2, SL_S2, SL_L2,
                           SL_Z2, SL_Q2, SL_Y2};
    block_partials<12>(acc, slots, partials, blockIdx.x);
  } else {
    double acc2[2] = {acc[0], acc[1]};
    const int slots[2] = {SL_QY, SL_YY};
    block_partials<2>(acc2, slots, partials, blockIdx.x);
  }
}

// PRO: the GLRED 2 final of the previous iteration (beta_i, alpha_i, the
// stopping test, the iteration count) runs in this kernel's prologue instead
// of a kernel of its own.  Every block loads the scalar struct and the GLRED 2
// partials (one memory round trip), reduces them with the fixed-order tree
// of block_sum_slots and runs the scalar logic on an LDS copy of the struct,
// so all blocks hold the same alpha_i, beta_i, omega_{i-1} and stopping
// decision.  The struct itself must not change while blocks may still read
// it, so block 0 writes the updated copy to the staging struct sc[1] (and
// the history row); phase B, which follows, reads its scalars from there and
// its block 0 commits sc[1] to sc[0].  Used without the automated criterion
// only (its 24 reduced slots are too many to load in every block).
template <typename T, int PC, bool NT, bool AUTO, int KIND, bool PRO>
__global__ __launch_bounds__(kBlock) void k_phaseA(PhaseAArgs<T> A, StParams<T> P, int64_t n,
                                                   DevScalars* __restrict__ sc,
                                                   double* __restrict__ partials, int64_t ntiles) {
  static_assert(!(PRO && AUTO), "the prologue final serves the periodic strategy only");
  // the first tile goes to LDS ahead of the prologue (cached streams only)
  constexpr bool PF = PRO && !NT;
  __shared__ __attribute__((aligned(16))) char pf[PF ? kPfBytes : 16];
  if constexpr (PF) {
    const auto first = tile_seq<KIND>(ntiles, V16<T>::n, P);
    if (first.valid() && first.has) phaseA_prefetch<T>(A, first.row(), pf);
  }
  // the scalars are loaded with the done flag (one round trip, not two)
  const int done = sc->done, n_saved = sc->n_saved;
  double alpha = sc->alpha, beta = sc->beta, omega_prev = sc->omega_prev;
  if constexpr (PRO) {
    // No early exit here: the prologue's loads (the GLRED 2 inputs and
    // partials) go out at once with the ones above, and every path uses
    // them, so none waits for the done test.  A stopped solve only copies
    // sc[0] to the staging struct.
    G2In in;
    in.done = done;
    in.omega = sc->omega; in.rho = sc->rho; in.tol = sc->tol; in.nb = sc->nb;
    in.its = sc->iter + 1; in.maxit = sc->maxit;
    const int sl[5] = {SL_RR0, SL_RW0, SL_RS0, SL_RZ0, SL_RR};
    slot_loads<5>(partials, sl, in.pp);
    if (!phaseA_prologue(sc, in, alpha, beta, omega_prev)) {
      if constexpr (PF) prefetch_wait();      // no LDS write may land after the block ends
      return;
    }
  } else {
    if (done) return;
  }
  if (n_saved)
    phaseA_body<T, PC, NT, AUTO, KIND, true, PF>(A, P, n, partials, ntiles, alpha, beta,
                                                  omega_prev, pf);
  else
    phaseA_body<T, PC, NT, AUTO, KIND, false, PF>(A, P, n, partials, ntiles, alpha, beta,
                                                   omega_prev, pf);
}

template <typename T>
struct PhaseBArgs {
  double* __restrict__ x;
  const T* __restrict__ g;
  const T* __restrict__ l;
  const T* __restrict__ s;
  const T* __restrict__ z;
  const T* __restrict__ t;
  T* __restrict__ v;                // read, or written when the product is fused
  const T* __restrict__ rhat;
  T* __restrict__ r;
  T* __restrict__ k;
  T* __restrict__ w;
  T* __restrict__ pm;               // m_{i+1} = M^-1 w_{i+1} for the next product, or null
  const T* __restrict__ dinv;
  T dinv_s;
};

// Phase B: with omega_i known,
//   u_i = k_i - alpha_i l_i,  q_i = r_i - alpha_i s_i,  y_i = w_i - alpha_i z_i
//   x_{i+1} = (x_i + alpha_i g_i) + omega_i u_i           (FP64)
//   r_{i+1} = q_i - omega_i y_i
//   k_{i+1} = u_i - omega_i (m_i - alpha_i n_i)           m_i = M^-1 w_i, n_i = M^-1 z_i
//   w_{i+1} = y_i - omega_i (t_i - alpha_i v_i)
// in place, and the GLRED 2 partials (r0, r_{i+1}), (r0, w_{i+1}), (r0, s_i),
// (r0, z_i), (r_{i+1}, r_{i+1}); AUTO adds ||x_i||^2, ||u_i||^2, ||n_i||^2, ||v_i||^2.
//
// KIND != 0 (a structured operator): v_i = A n_i = A M^-1 z_i is computed
// here from z_i, final since phase A, instead of being read (the SPMV that
// the unfused iteration runs between the phases), and stored for the next
// phase A; z is read with cached loads for the neighbours' sake.  With no
// SPMV kernel between the phases to carry it, the GLRED 1 final runs in
// this kernel's prologue.
// Registers of one phase B chunk
template <typename T>
struct BTile {
  static constexpr int C = V16<T>::n;
  T g[C], l[C], s[C], z[C], t[C], v[C], rh[C], r[C], k[C], w[C], d[C], n[C];
  double x[C];
  T pd[C], pu[C];     // plane march, 3D: z a plane below and above (as stored)
};

// the loads of one chunk
template <typename T, int PC, bool NT, int KIND>
__device__ __forceinline__ void phaseB_issue(const PhaseBArgs<T>& B, int64_t i, BTile<T>& R,
                                             bool have_z = false) {
  constexpr int C = V16<T>::n;
  constexpr bool FUSE = KIND != 0;
  ldc<T, C, NT>(B.g + i, R.g); ldc<T, C, NT>(B.l + i, R.l); ldc<T, C, NT>(B.s + i, R.s);
  if (!have_z) ldc<T, C, NT && !FUSE>(B.z + i, R.z);
  ldc<T, C, NT>(B.t + i, R.t);
  if (!FUSE) ldc<T, C, NT>(B.v + i, R.v);
  ldc<T, C, NT>(B.rhat + i, R.rh); ldc<T, C, NT>(B.r + i, R.r); ldc<T, C, NT>(B.k + i, R.k);
  ldc<T, C, NT>(B.w + i, R.w);
  ldc<double, C, NT>(B.x + i, R.x);
  if (PC == PC_VECTOR) ldc<T, C, NT>(B.dinv + i, R.d);
}

// n = M^-1 z of one chunk and, fused, v = A n from the neighbours of z
template <typename T, int PC, int KIND, bool NT>
__device__ __forceinline__ void phaseB_stencil(const PhaseBArgs<T>& B, const StParams<T>& P,
                                               int64_t nrows, int64_t i, BTile<T>& R) {
  constexpr int C = V16<T>::n;
#pragma unroll
  for (int e = 0; e < C; ++e) {
    const T de = (PC == PC_VECTOR) ? R.d[e] : B.dinv_s;
    R.n[e] = (PC == PC_NONE) ? R.z[e] : de * R.z[e];
  }
  if constexpr (KIND != 0) {
    if (march_fused<KIND, PC>(P)) {
      T xd[C], xu[C];
#pragma unroll
      for (int e = 0; e < C; ++e) {
        xd[e] = prec1<T, PC>(R.pd[e], nullptr, B.dinv_s, 0);
        xu[e] = prec1<T, PC>(R.pu[e], nullptr, B.dinv_s, 0);
      }
      st_apply3_planes<T, PC>(P, B.z, B.dinv, B.dinv_s, (int)i, xd, R.n, xu, R.v);
    } else if (i < nrows) {
      st_apply<T, PC, KIND, 1, NT && sizeof(T) == 8>(P, B.z, B.dinv, B.dinv_s, (int)i, R.n,
                                                     R.v);
    } else {
#pragma unroll
      for (int e = 0; e < C; ++e) R.v[e] = T(0);          // padding rows stay zero
    }
  }
}

// the updates of one chunk and their partials
template <typename T, int PC, bool NT, bool AUTO, int KIND>
__device__ __forceinline__ void phaseB_update(const PhaseBArgs<T>& B, int64_t i, BTile<T>& R,
                                              double alpha, double omega, double (&acc)[9]) {
  constexpr int C = V16<T>::n;
  constexpr bool FUSE = KIND != 0;
  const T a = (T)alpha, om = (T)omega;
#pragma unroll
  for (int e = 0; e < C; ++e) {
    const T de = (PC == PC_VECTOR) ? R.d[e] : B.dinv_s;
    const T m = (PC == PC_NONE) ? R.w[e] : de * R.w[e];
    const T q = R.r[e] - a * R.s[e];
    const T u = R.k[e] - a * R.l[e];
    const T y = R.w[e] - a * R.z[e];
    if (AUTO) {
      acc[5] += R.x[e] * R.x[e];
      acc[6] += (double)u * (double)u;
      acc[7] += (double)R.n[e] * (double)R.n[e];
      acc[8] += (double)R.v[e] * (double)R.v[e];
    }
    R.x[e] = (R.x[e] + alpha * (double)R.g[e]) + omega * (double)u;
    const T rn = q - om * y;
    const T kn = u - om * (m - a * R.n[e]);
    const T wn = y - om * (R.t[e] - a * R.v[e]);
    R.r[e] = rn; R.k[e] = kn; R.w[e] = wn;
    const double rhd = (double)R.rh[e];
    acc[0] += rhd * (double)rn;
    acc[1] += rhd * (double)wn;
    acc[2] += rhd * (double)R.s[e];
    acc[3] += rhd * (double)R.z[e];
    acc[4] += (double)rn * (double)rn;
  }
  stc<T, C, NT>(B.r + i, R.r); stc<T, C, NT>(B.k + i, R.k); stc<T, C, NT>(B.w + i, R.w);
  stc<double, C, NT>(B.x + i, R.x);
  if (FUSE) stc<T, C, NT>(B.v + i, R.v);
  if constexpr (!FUSE && PC == PC_VECTOR) {
    if (B.pm) {                       // m_{i+1} = M^-1 w_{i+1}, the next product's input
      T pw[C];
#pragma unroll
      for (int e = 0; e < C; ++e) pw[e] = R.d[e] * R.w[e];
      stc<T, C, NT>(B.pm + i, pw);
    }
  }
}

// STAGED: phase A ran the previous GLRED 2 final in its prologue and left
// the updated scalars in sc[1]; they are read from there, and block 0
// commits them to sc[0] before it records omega.
template <typename T, int PC, bool NT, bool AUTO, int KIND, bool STAGED>
__global__ __launch_bounds__(kBlock) void k_phaseB(PhaseBArgs<T> B, StParams<T> P, int64_t nrows,
                                                   DevScalars* __restrict__ sc,
                                                   double* __restrict__ partials, int64_t ntiles) {
  constexpr int C = V16<T>::n;
  const DevScalars* in = STAGED ? sc + 1 : sc;
  const int done = in->done;
  const double alpha = in->alpha;
  double omega = in->omega;
  if (STAGED && blockIdx.x == 0) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(sc + 1);
    uint32_t* dst = reinterpret_cast<uint32_t*>(sc);
    for (int i = threadIdx.x; i < kScWords; i += kBlock) dst[i] = src[i];
    __syncthreads();
  }
  if (done) return;
  auto it = tile_seq<KIND>(ntiles, C, P);
  const bool mw = march_fused<KIND, PC>(P);      // fused 3D product, planes in registers
  BTile<T> R;
  const bool any = it.valid() && it.has;
  // The first chunk's loads do not depend on omega: they go out together
  // with the loads of the GLRED 1 partials (one memory round trip for both).
  if (any) {
    phaseB_issue<T, PC, NT, KIND>(B, it.row(), R);
    if constexpr (marchable<KIND>()) if (mw) march_planes<T>(B.z, it, R.pd, R.pu);
  }
  if constexpr (KIND != 0) {
    // GLRED 1 final (omega_i = (q_i, y_i) / (y_i, y_i)), reduced by every
    // block from phase A's partials with the fixed-order tree of
    // block_sum_slots, so all blocks hold the same omega; block 0 records
    // it.  This kernel writes only GLRED 2 slots, so the GLRED 1 partials
    // stay intact while it runs.
    const int sl[2] = {SL_QY, SL_YY};
    double pp[2][kSlotStrides], ts[2], v[2];
    slot_loads<2>(partials, sl, pp);
    if (any) phaseB_stencil<T, PC, KIND, NT>(B, P, nrows, it.row(), R);
    slot_thread_sums<2>(pp, gridDim.x, ts);
    block_tree<2>(ts, v);
    const bool bad = !finite(v[0]) || !finite(v[1]);
    omega = v[1] != 0.0 ? v[0] / v[1] : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->sig[SL_QY] = v[0];
      sc->sig[SL_YY] = v[1];
      sc->n_saved = 0;                 // phase A of this iteration has consumed it
      if (bad) stop(sc, ST_NONFINITE);
      else sc->omega = omega;
    }
    if (bad) return;
  } else {
    if (any) phaseB_stencil<T, PC, KIND, NT>(B, P, nrows, it.row(), R);
  }
  double acc[9];
#pragma unroll
  for (int d = 0; d < 9; ++d) acc[d] = 0.0;
  while (it.valid()) {
    if (it.has) phaseB_update<T, PC, NT, AUTO, KIND>(B, it.row(), R, alpha, omega, acc);
    it.next();
    if (it.valid() && it.has) {
      const bool carry = mw && it.cont;
      if (carry) march_rotate<T>(R.z, R.pd, R.pu);
      phaseB_issue<T, PC, NT, KIND>(B, it.row(), R, carry);
      if constexpr (marchable<KIND>()) if (mw) march_planes<T>(B.z, it, R.pd, R.pu);
      phaseB_stencil<T, PC, KIND, NT>(B, P, nrows, it.row(), R);
    }
  }
  if (AUTO) {
    const int slots[9] = {SL_RR0, SL_RW0, SL_RS0, SL_RZ0, SL_RR, SL_X2, SL_U2, SL_N2, SL_V2};
    block_partials<9>(acc, slots, partials, blockIdx.x);
  } else {
    double acc5[5] = {acc[0], acc[1], acc[2], acc[3], acc[4]};
    const int slots[5] = {SL_RR0, SL_RW0, SL_RS0, SL_RZ0, SL_RR};
    block_partials<5>(acc5, slots, partials, blockIdx.x);
  }
}

// Classic BiCGStab (Algorithm 1) vector update, with alpha_i and omega_i known:
//   q_i = r_i - alpha_i s_i, g_i = M^-1 p_i, u_i = M^-1 q_i
//   x_{i+1} = (x_i + alpha_i g_i) + omega_i u_i,  r_{i+1} = q_i - omega_i y_i
// and the third reduction's partials (r0, r_{i+1}), (r_{i+1}, r_{i+1}).
template <typename T>
struct ClUpdArgs {
  double* __restrict__ x;
  const T* __restrict__ p;
  const T* __restrict__ s;
  const T* __restrict__ y;
  const T* __restrict__ rhat;
  T* __restrict__ r;
  const T* __restrict__ dinv;
  T dinv_s;
};

template <typename T, int PC>
__global__ __launch_bounds__(kBlock) void k_cl_update(ClUpdArgs<T> U, const DevScalars* __restrict__ sc,
                                                      double* __restrict__ partials, int64_t ntiles) {
  const int done = sc->done;
  const double alpha = sc->alpha, omega = sc->omega;
  if (done) return;
  constexpr int W = V16<T>::n;
  const T a = (T)alpha, om = (T)omega;
  double acc[2] = {0.0, 0.0};
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t i = (tile * kBlock + threadIdx.x) * W;
    T p[W], s[W], y[W], rh[W], r[W], d[W];
    double x[W];
    ld16(U.p + i, p); ld16(U.s + i, s); ld16(U.y + i, y); ld16(U.rhat + i, rh); ld16(U.r + i, r);
#pragma unroll
    for (int h = 0; h < W; h += 2) {
      double xx[2];
      ld16(U.x + i + h, xx);
      x[h] = xx[0]; x[h + 1] = xx[1];
    }
    if (PC == PC_VECTOR) ld16(U.dinv + i, d);
#pragma unroll
    for (int e = 0; e < W; ++e) {
      const T de = (PC == PC_VECTOR) ? d[e] : U.dinv_s;
      const T q = r[e] - a * s[e];
      const T g = (PC == PC_NONE) ? p[e] : de * p[e];
      const T u = (PC == PC_NONE) ? q : de * q;
      x[e] = (x[e] + alpha * (double)g) + omega * (double)u;
      const T rn = q - om * y[e];
      r[e] = rn;
      acc[0] += (double)rh[e] * (double)rn;
      acc[1] += (double)rn * (double)rn;
    }
    st16(U.r + i, r);
#pragma unroll
    for (int h = 0; h < W; h += 2) {
      double xx[2] = {x[h], x[h + 1]};
      st16(U.x + i + h, xx);
    }
  }
  const int slots[2] = {SL_RR0, SL_RR};
  block_partials<2>(acc, slots, partials, blockIdx.x);
}

// Classic: p_{i+1} = r_{i+1} + beta_i (p_i - omega_i s_i)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cl_p(const T* __restrict__ r, T* __restrict__ p,
                                                 const T* __restrict__ s,
                                                 const DevScalars* __restrict__ sc, int64_t ntiles) {
  const int done = sc->done;
  const double beta = sc->beta, omega = sc->omega;
  if (done) return;
  constexpr int W = V16<T>::n;
  const T b = (T)beta, om = (T)omega;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t i = (tile * kBlock + threadIdx.x) * W;
    T rr[W], pp[W], ss[W];
    ld16(r + i, rr); ld16(p + i, pp); ld16(s + i, ss);
#pragma unroll
    for (int e = 0; e < W; ++e) pp[e] = rr[e] + b * (pp[e] - om * ss[e]);
    st16(p + i, pp);
  }
}

template <int NS>
__global__ __launch_bounds__(kBlock) void k_final(int mode, FinSlots fs, DevScalars* __restrict__ sc,
                                                  const double* __restrict__ partials, int nblk,
                                                  int aux, int respect_done) {
  one_block_final<NS>(mode, fs, sc, partials, nblk, aux, respect_done != 0);
}

template <typename T>
__global__ void k_fill_zero(T* __restrict__ p, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = T(0);
}

template <typename T>
__global__ void k_to_double(const T* __restrict__ src, double* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (double)src[i];
}

// plain FP64 copy with the same tiling as the phase kernels (bandwidth calibration)
__global__ __launch_bounds__(kBlock) void k_copy(const double* __restrict__ src,
                                                 double* __restrict__ dst, int64_t ntiles) {
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t i = (tile * kBlock + threadIdx.x) * 2;
    double v[2];
    ld16(src + i, v);
    st16(dst + i, v);
  }
}

void launch_copy(Solver& S, const double* src, double* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_copy, dim3(S.nblk), dim3(kBlock), 0, st, src, dst, S.npad / (kBlock * 2));
}

// The products reading of the gap bound f^r (Section 3.6): the moduli of the
// entries of the products of the error propagation matrices of
// eq:all_error_matrices that carry each group of local errors into the
// residual gap (R through U; S through BA; W through UEA and UC; Z through
// BAEA, BPA, BAC and BD, with A, B, C, D, E, P, U of eq:all_matrices built
// from the signed alpha, beta, omega), times the bound of the group.  The
// state is one row per source j of local errors: the current column of the
// twelve partial products and the four group bounds.  Every update is
// elementwise in j: a product ending in A, C or D gains its left factor's
// column times -alpha_c, -omega_c or omega_c alpha_c; one ending in B, E or
// P is scaled by beta_{c+1} and gains the left factor's new column (B, E) or
// its old column times -omega_c (P).  The A/C/D step needs alpha_c, omega_c
// only, so f^r_{c+1} is known at the end of iteration c; the B/E/P step waits
// for beta_{c+1}, which the next iteration's final brings.  Column 0 holds
// the initial gaps (Section 3.2); R and W sources of iteration c sit in row
// c+1, S and Z sources in row c.  A replacement starts a new system whose
// row 0 holds the recomputed s and z gaps and row 1 the recomputed r and w
// gaps (alpha_0 = 0).  One block; the sum over the rows uses a fixed tree.
constexpr int kProdThreads = 1024;
enum : int {
  PB_B = 0, PB_BA, PB_BD, PB_BAC, PB_BAE, PB_BAEA, PB_BP, PB_BPA, PB_U, PB_UE, PB_UEA, PB_UC,
  PB_TR, PB_TS, PB_TW, PB_TZ, PB_COUNT
};

__global__ __launch_bounds__(kProdThreads) void k_bound_products(DevScalars* __restrict__ sc) {
  __shared__ double wsum[kProdThreads / 64];
  const int op = sc->pr_op;
  if (op == 0) return;
  double* __restrict__ st = sc->pr_state;
  const int64_t cap = sc->pr_cap;
  int64_t c = sc->pr_c;
  int first = sc->pr_first, pending = sc->pr_pending;
  const double fr_in = sc->fr, dw_in = sc->dw;
  const int tid = threadIdx.x;
  __syncthreads();                        // every thread has read the state
  double f = fr_in;
  if (op & PR_RESET) {
    // a new system: row 0 the recomputed s, z gaps; row 1 the recomputed r, w
    // gaps, entering with the leading alpha_0 = 0 step
    if (tid < 2) {
      for (int k = 0; k < PB_COUNT; ++k) st[k * cap + tid] = 0.0;
      st[PB_U * cap + tid] = 1.0;
      if (tid == 0) {
        st[PB_B * cap] = 1.0;
        st[PB_TS * cap] = sc->pr_rS;
        st[PB_TZ * cap] = sc->pr_rZ;
      } else {
        st[PB_TR * cap + 1] = sc->pr_rR;
        st[PB_TW * cap + 1] = sc->pr_rW;
      }
    }
    c = 0; first = 0; pending = 1;
    f = sc->pr_rR;
  } else if (op & PR_START) {
    if (tid == 0) {
      for (int k = 0; k < PB_COUNT; ++k) st[k * cap] = 0.0;
      st[PB_B * cap] = 1.0;
      st[PB_U * cap] = 1.0;
      st[PB_TR * cap] = fr_in;             // ||Delta^r_0|| and ||Delta^w_0||
      st[PB_TW * cap] = dw_in;
    }
    c = 0; first = 1; pending = 0;
    f = fr_in;
  } else if (op & PR_STEP) {
    const double a = sc->pr_a, b = sc->pr_b, w = sc->pr_w, wp = sc->pr_wp;
    const double tSc = first ? sc->pr_S0 : sc->pr_S, tZc = first ? sc->pr_Z0 : sc->pr_Z;
    const double tRn = sc->pr_R, tWn = sc->pr_W;
    const bool ebp = !first && pending;
    const int64_t cn = ebp ? c + 1 : c;    // the column of this step's S and Z sources
    double acc = 0.0;
    for (int64_t j = tid; j <= cn + 1; j += kProdThreads) {
      if (j == cn + 1) {                   // the new row: this step's R and W sources
        for (int k = 0; k < PB_COUNT; ++k) st[k * cap + j] = 0.0;
        st[PB_U * cap + j] = 1.0;
        st[PB_TR * cap + j] = tRn;
        st[PB_TW * cap + j] = tWn;
        acc += tRn;
        continue;
      }
      double v[PB_COUNT];
#pragma unroll
      for (int k = 0; k < PB_COUNT; ++k) v[k] = st[k * cap + j];
      if (ebp) {                           // column c -> c+1 of the B, E, P products
        v[PB_BP] = b * (v[PB_BP] - wp * v[PB_B]);
        v[PB_B] = j == cn ? 1.0 : b * v[PB_B];
        v[PB_BAE] = b * v[PB_BAE] + v[PB_BA];
        v[PB_UE] = b * v[PB_UE] + v[PB_U];
      }
      if (j == cn) {
        v[PB_TS] = tSc;
        v[PB_TZ] = tZc;
      }
      const double ba = v[PB_BA];          // column cn -> cn+1 of the A, C, D products
      v[PB_BA] = ba - a * v[PB_B];
      v[PB_BD] = v[PB_BD] + w * a * v[PB_B];
      v[PB_BAC] = v[PB_BAC] - w * ba;
      v[PB_BAEA] = v[PB_BAEA] - a * v[PB_BAE];
      v[PB_BPA] = v[PB_BPA] - a * v[PB_BP];
      v[PB_UEA] = v[PB_UEA] - a * v[PB_UE];
      v[PB_UC] = v[PB_UC] - w * v[PB_U];
#pragma unroll
      for (int k = 0; k < PB_COUNT; ++k) st[k * cap + j] = v[k];
      acc += v[PB_TR] + v[PB_TS] * fabs(v[PB_BA]) +
             v[PB_TW] * (fabs(v[PB_UEA]) + fabs(v[PB_UC])) +
             v[PB_TZ] * (fabs(v[PB_BAEA]) + fabs(v[PB_BPA]) + fabs(v[PB_BAC]) + fabs(v[PB_BD]));
    }
    acc = wave_sum(acc);
    if ((tid & 63) == 0) wsum[tid >> 6] = acc;
    __syncthreads();
    f = 0.0;
    for (int k = 0; k < kProdThreads / 64; ++k) f += wsum[k];
    c = cn; first = 0; pending = 1;
  }
  if (tid == 0) {
    sc->pr_c = (int32_t)c;
    sc->pr_first = first;
    sc->pr_pending = pending;
    sc->fr = f;
    const int its = sc->pr_its;
    if ((op & (PR_STEP | PR_RESET)) && sc->bound_history && its >= 1 && its <= sc->bound_len)
      sc->bound_history[its - 1] = f;
    if (op & PR_CRIT) {                    // eq:criterion for the next step
      const int f_ok = f <= sc->tau * sc->pr_rn;
      sc->rr_next = sc->f_ok_prev && !f_ok;
      sc->f_ok_prev = f_ok;
    }
    sc->pr_op = 0;
  }
}

void launch_bound_products(Solver& S, hipStream_t st) {
  if (!S.bound_prod) return;
  hipLaunchKernelGGL(k_bound_products, dim3(1), dim3(kProdThreads), 0, st, S.sc);
}

__global__ void k_set_done(DevScalars* sc, int value) {
  if (threadIdx.x == 0 && blockIdx.x == 0) sc->done = value;
}

// ----------------------------------------------------------------------------
// launchers
// ----------------------------------------------------------------------------

static inline int fill_blocks(int64_t count) {
  int64_t b = (count + kBlock - 1) / kBlock;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (int)b;
}

// Launches kern<KIND> for the fused operator kind (0: none).  Only the
// kinds that fused_kind() can return for this preconditioner are
// instantiated: constant stencils with a scalar Jacobi scale, DIA5 with a
// Jacobi vector, either without a preconditioner.
template <int PC, class F>
static void with_fused_kind(int kind, F&& f) {
  if (kind == OP_ST2D5) {
    if constexpr (PC != PC_VECTOR) { f(std::integral_constant<int, OP_ST2D5>{}); return; }
  } else if (kind == OP_ST3D7) {
    if constexpr (PC != PC_VECTOR) { f(std::integral_constant<int, OP_ST3D7>{}); return; }
  } else if (kind == OP_DIA5) {
    if constexpr (PC != PC_SCALAR) { f(std::integral_constant<int, OP_DIA5>{}); return; }
  } else {
    f(std::integral_constant<int, 0>{});
    return;
  }
  throw std::logic_error("fused operator kind without a phase kernel");
}

template <typename T, int PC>
static void phaseA_t(Solver& S, bool tr, bool pro, hipStream_t st) {
  PhaseAArgs<T> a;
  a.k = (const T*)S.vec[V_K]; a.w = (const T*)S.vec[V_W]; a.t = (T*)S.vec[V_T];
  a.r = (const T*)S.vec[V_R]; a.v = (const T*)S.vec[V_V];
  a.g = (T*)S.vec[V_G]; a.s = (T*)S.vec[V_S]; a.l = (T*)S.vec[V_L]; a.z = (T*)S.vec[V_Z];
  a.zsave = (const T*)S.vec[V_TMP];
  a.pm = pre_multiplied(S, tr) ? (T*)S.vec[V_PM] : nullptr;
  a.dinv = (const T*)S.dinv; a.dinv_s = (T)S.dinv_s;
  const int kind = fused_kind(S, tr);
  StParams<T> P = st_params<T>(S, op_of(S, tr));
  P.mz = phase_march_planes(S, tr);
  const int64_t nt = S.npad / (kBlock * V16<T>::n);
  const bool ntm = (S.vnt & 1) != 0;
  with_fused_kind<PC>(kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(S.nblk), dim3(kBlock), 0, st, a, P, S.n, S.sc, S.partials, nt);
    };
    if (S.auto_rr) {
      if (ntm) go(k_phaseA<T, PC, true, true, K, false>);
      else go(k_phaseA<T, PC, false, true, K, false>);
    } else if (pro) {
      if constexpr (K != 0) {
        if (ntm) go(k_phaseA<T, PC, true, false, K, true>);
        else go(k_phaseA<T, PC, false, false, K, true>);
      } else {
        throw std::logic_error("GLRED 2 prologue without a fused operator");
      }
    } else {
      if (ntm) go(k_phaseA<T, PC, true, false, K, false>);
      else go(k_phaseA<T, PC, false, false, K, false>);
    }
  });
}

template <typename T, int PC>
static void phaseB_t(Solver& S, bool tr, bool staged, hipStream_t st) {
  PhaseBArgs<T> a;
  a.x = S.x;
  a.g = (const T*)S.vec[V_G]; a.l = (const T*)S.vec[V_L]; a.s = (const T*)S.vec[V_S];
  a.z = (const T*)S.vec[V_Z]; a.t = (const T*)S.vec[V_T]; a.v = (T*)S.vec[V_V];
  a.rhat = (const T*)S.vec[V_RHAT];
  a.r = (T*)S.vec[V_R]; a.k = (T*)S.vec[V_K]; a.w = (T*)S.vec[V_W];
  a.pm = pre_multiplied(S, tr) ? (T*)S.vec[V_PM] : nullptr;
  a.dinv = (const T*)S.dinv; a.dinv_s = (T)S.dinv_s;
  const int kind = fused_kind(S, tr);
  StParams<T> P = st_params<T>(S, op_of(S, tr));
  P.mz = phase_march_planes(S, tr);
  const int64_t nt = S.npad / (kBlock * V16<T>::n);
  const bool ntm = (S.vnt & 2) != 0;
  with_fused_kind<PC>(kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(S.nblk), dim3(kBlock), 0, st, a, P, S.n, S.sc, S.partials, nt);
    };
    if (S.auto_rr) {
      if (ntm) go(k_phaseB<T, PC, true, true, K, false>);
      else go(k_phaseB<T, PC, false, true, K, false>);
    } else if (staged) {
      if constexpr (K != 0) {
        if (ntm) go(k_phaseB<T, PC, true, false, K, true>);
        else go(k_phaseB<T, PC, false, false, K, true>);
      } else {
        throw std::logic_error("staged scalars without a fused operator");
      }
    } else {
      if (ntm) go(k_phaseB<T, PC, true, false, K, false>);
      else go(k_phaseB<T, PC, false, false, K, false>);
    }
  });
}

template <typename T, int PC>
static void clupd_t(Solver& S, hipStream_t st) {
  ClUpdArgs<T> a;
  a.x = S.x;
  a.p = (const T*)S.vec[V_G]; a.s = (const T*)S.vec[V_S]; a.y = (const T*)S.vec[V_V];
  a.rhat = (const T*)S.vec[V_RHAT]; a.r = (T*)S.vec[V_R];
  a.dinv = (const T*)S.dinv; a.dinv_s = (T)S.dinv_s;
  hipLaunchKernelGGL((k_cl_update<T, PC>), dim3(S.nblk), dim3(kBlock), 0, st, a, S.sc,
                     S.partials, S.vtiles);
}

#define PBCG_DISPATCH_T_PC(S, FN, ...)                                      \
  do {                                                                      \
    if ((S).precision == 0) {                                               \
      if ((S).pc == PC_NONE) FN<double, PC_NONE>(__VA_ARGS__);              \
      else if ((S).pc == PC_SCALAR) FN<double, PC_SCALAR>(__VA_ARGS__);     \
      else FN<double, PC_VECTOR>(__VA_ARGS__);                              \
    } else {                                                                \
      if ((S).pc == PC_NONE) FN<float, PC_NONE>(__VA_ARGS__);               \
      else if ((S).pc == PC_SCALAR) FN<float, PC_SCALAR>(__VA_ARGS__);      \
      else FN<float, PC_VECTOR>(__VA_ARGS__);                               \
    }                                                                       \
  } while (0)

void launch_phaseA(Solver& S, bool tr, bool pro, hipStream_t st) {
  PBCG_DISPATCH_T_PC(S, phaseA_t, S, tr, pro, st);
}
void launch_phaseB(Solver& S, bool tr, bool staged, hipStream_t st) {
  PBCG_DISPATCH_T_PC(S, phaseB_t, S, tr, staged, st);
}
void launch_cl_update(Solver& S, hipStream_t st) { PBCG_DISPATCH_T_PC(S, clupd_t, S, st); }

void launch_cl_p(Solver& S, hipStream_t st) {
  if (S.precision == 0)
    hipLaunchKernelGGL(k_cl_p<double>, dim3(S.nblk), dim3(kBlock), 0, st,
                       (const double*)S.vec[V_R], (double*)S.vec[V_G], (const double*)S.vec[V_S],
                       S.sc, S.vtiles);
  else
    hipLaunchKernelGGL(k_cl_p<float>, dim3(S.nblk), dim3(kBlock), 0, st,
                       (const float*)S.vec[V_R], (float*)S.vec[V_G], (const float*)S.vec[V_S],
                       S.sc, S.vtiles);
}

void launch_final(Solver& S, int mode, int aux, hipStream_t st, bool force) {
  const int respect = (force || mode == FIN_TRUE || mode == FIN_SUM || mode == FIN_INIT ||
                       mode == FIN_C_INIT || mode == FIN_REDO) ? 0 : 1;
  const FinSlots fs = fin_slots(mode, S.auto_rr ? 1 : 0, aux);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(1), dim3(kBlock), 0, st, mode, fs, S.sc, S.partials, S.nblk,
                       aux, respect);
  };
  // the smallest instantiated slot count that holds the mode's slots
  if (fs.n <= 1) go(k_final<1>);
  else if (fs.n <= 2) go(k_final<2>);
  else if (fs.n <= 5) go(k_final<5>);
  else if (fs.n <= 8) go(k_final<8>);
  else go(k_final<kMaxFinSlots>);
}

void launch_fill_zero(Solver& S, void* ptr, int64_t count, size_t elem, hipStream_t st) {
  (void)S;
  if (count <= 0) return;
  if (elem == 8)
    hipLaunchKernelGGL(k_fill_zero<double>, dim3(fill_blocks(count)), dim3(kBlock), 0, st,
                       (double*)ptr, count);
  else
    hipLaunchKernelGGL(k_fill_zero<float>, dim3(fill_blocks(count)), dim3(kBlock), 0, st,
                       (float*)ptr, count);
}

void launch_to_double(Solver& S, const void* src, double* dst, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  if (S.precision == 0)
    hipLaunchKernelGGL(k_to_double<double>, dim3(fill_blocks(n)), dim3(kBlock), 0, st,
                       (const double*)src, dst, n);
  else
    hipLaunchKernelGGL(k_to_double<float>, dim3(fill_blocks(n)), dim3(kBlock), 0, st,
                       (const float*)src, dst, n);
}

void launch_set_done(Solver& S, int value, hipStream_t st) {
  hipLaunchKernelGGL(k_set_done, dim3(1), dim3(64), 0, st, S.sc, value);
}

}  // namespace pbcg
