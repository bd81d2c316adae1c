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
template <typename T, int PC, bool NT, bool AUTO, int KIND, bool SAVED>
__device__ __forceinline__ void phaseA_body(const PhaseAArgs<T>& A, const StParams<T>& P,
                                            int64_t n, T a, T b, T wp, double (&acc)[12],
                                            int64_t ntiles) {
  constexpr int C = V16<T>::n;
  constexpr bool FUSE = KIND != 0;
  for (XcdWalk it(ntiles, blockIdx.x, gridDim.x); it.t < it.end; it.t += it.step) {
    const int64_t i = (it.t * kBlock + threadIdx.x) * C;
    T k[C], w[C], t[C], r[C], v[C], g[C], s[C], l[C], z[C], zp[C], d[C], m[C];
    ldc<T, C, NT>(A.k + i, k); ldc<T, C, NT && !FUSE>(A.w + i, w);
    if (!FUSE) ldc<T, C, NT>(A.t + i, t);
    ldc<T, C, NT>(A.r + i, r); ldc<T, C, NT>(A.v + i, v); ldc<T, C, NT>(A.g + i, g);
    ldc<T, C, NT>(A.s + i, s); ldc<T, C, NT>(A.l + i, l); ldc<T, C, NT>(A.z + i, z);
    if (SAVED) ldc<T, C, NT>(A.zsave + i, zp);
    if (PC == PC_VECTOR) ldc<T, C, NT>(A.dinv + i, d);
#pragma unroll
    for (int e = 0; e < C; ++e) {
      const T de = (PC == PC_VECTOR) ? d[e] : A.dinv_s;
      m[e] = (PC == PC_NONE) ? w[e] : de * w[e];
    }
    if constexpr (FUSE) {
      if (i < n) {
        st_apply<T, PC, KIND, 1>(P, A.w, A.dinv, A.dinv_s, (int)i, m, t);
      } else {
#pragma unroll
        for (int e = 0; e < C; ++e) t[e] = T(0);          // padding rows stay zero
      }
    }
#pragma unroll
    for (int e = 0; e < C; ++e) {
      const T de = (PC == PC_VECTOR) ? d[e] : A.dinv_s;
      const T zprev = SAVED ? zp[e] : z[e];
      const T np = (PC == PC_NONE) ? zprev : de * zprev;
      const T gn = k[e] + b * (g[e] - wp * l[e]);
      const T sn = w[e] + b * (s[e] - wp * z[e]);
      const T ln = m[e] + b * (l[e] - wp * np);
      const T zn = t[e] + b * (z[e] - wp * v[e]);
      const T q = r[e] - a * sn;
      const T y = w[e] - a * zn;
      acc[0] += (double)q * (double)y;
      acc[1] += (double)y * (double)y;
      if (AUTO) {
        acc[2] += (double)k[e] * (double)k[e];
        acc[3] += (double)w[e] * (double)w[e];
        acc[4] += (double)t[e] * (double)t[e];
        acc[5] += (double)m[e] * (double)m[e];
        acc[6] += (double)gn * (double)gn;
        acc[7] += (double)sn * (double)sn;
        acc[8] += (double)ln * (double)ln;
        acc[9] += (double)zn * (double)zn;
        acc[10] += (double)q * (double)q;
        acc[11] += (double)y * (double)y;
      }
      g[e] = gn; s[e] = sn; l[e] = ln; z[e] = zn;
    }
    stc<T, C, NT>(A.g + i, g); stc<T, C, NT>(A.s + i, s); stc<T, C, NT>(A.l + i, l);
    stc<T, C, NT>(A.z + i, z);
    if (FUSE) stc<T, C, NT>(A.t + i, t);
  }
}

template <typename T, int PC, bool NT, bool AUTO, int KIND>
__global__ __launch_bounds__(kBlock) void k_phaseA(PhaseAArgs<T> A, StParams<T> P, int64_t n,
                                                   const DevScalars* __restrict__ sc,
                                                   double* __restrict__ partials, int64_t ntiles) {
  // the scalars are loaded with the done flag (one round trip, not two)
  const int done = sc->done, n_saved = sc->n_saved;
  const double alpha = sc->alpha, beta = sc->beta, omega_prev = sc->omega_prev;
  if (done) return;
  const T a = (T)alpha, b = (T)beta, wp = (T)omega_prev;
  double acc[12];
#pragma unroll
  for (int d = 0; d < 12; ++d) acc[d] = 0.0;
  if (n_saved) phaseA_body<T, PC, NT, AUTO, KIND, true>(A, P, n, a, b, wp, acc, ntiles);
  else phaseA_body<T, PC, NT, AUTO, KIND, false>(A, P, n, a, b, wp, acc, ntiles);
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
// phase A; z is read with cached loads for the neighbours' sake.
template <typename T, int PC, bool NT, bool AUTO, int KIND>
__global__ __launch_bounds__(kBlock) void k_phaseB(PhaseBArgs<T> B, StParams<T> P, int64_t nrows,
                                                   const DevScalars* __restrict__ sc,
                                                   double* __restrict__ partials, int64_t ntiles) {
  const int done = sc->done;
  const double alpha = sc->alpha, omega = sc->omega;
  if (done) return;
  constexpr int C = V16<T>::n;
  constexpr bool FUSE = KIND != 0;
  const T a = (T)alpha, om = (T)omega;
  double acc[9];
#pragma unroll
  for (int d = 0; d < 9; ++d) acc[d] = 0.0;
  for (XcdWalk it(ntiles, blockIdx.x, gridDim.x); it.t < it.end; it.t += it.step) {
    const int64_t i = (it.t * kBlock + threadIdx.x) * C;
    T g[C], l[C], s[C], z[C], t[C], v[C], rh[C], r[C], k[C], w[C], d[C], n[C];
    double x[C];
    ldc<T, C, NT>(B.g + i, g); ldc<T, C, NT>(B.l + i, l); ldc<T, C, NT>(B.s + i, s);
    ldc<T, C, NT && !FUSE>(B.z + i, z); ldc<T, C, NT>(B.t + i, t);
    if (!FUSE) ldc<T, C, NT>(B.v + i, v);
    ldc<T, C, NT>(B.rhat + i, rh); ldc<T, C, NT>(B.r + i, r); ldc<T, C, NT>(B.k + i, k);
    ldc<T, C, NT>(B.w + i, w);
    ldc<double, C, NT>(B.x + i, x);
    if (PC == PC_VECTOR) ldc<T, C, NT>(B.dinv + i, d);
#pragma unroll
    for (int e = 0; e < C; ++e) {
      const T de = (PC == PC_VECTOR) ? d[e] : B.dinv_s;
      n[e] = (PC == PC_NONE) ? z[e] : de * z[e];
    }
    if constexpr (FUSE) {
      if (i < nrows) {
        st_apply<T, PC, KIND, 1>(P, B.z, B.dinv, B.dinv_s, (int)i, n, v);
      } else {
#pragma unroll
        for (int e = 0; e < C; ++e) v[e] = T(0);          // padding rows stay zero
      }
    }
#pragma unroll
    for (int e = 0; e < C; ++e) {
      const T de = (PC == PC_VECTOR) ? d[e] : B.dinv_s;
      const T m = (PC == PC_NONE) ? w[e] : de * w[e];
      const T q = r[e] - a * s[e];
      const T u = k[e] - a * l[e];
      const T y = w[e] - a * z[e];
      if (AUTO) {
        acc[5] += x[e] * x[e];
        acc[6] += (double)u * (double)u;
        acc[7] += (double)n[e] * (double)n[e];
        acc[8] += (double)v[e] * (double)v[e];
      }
      x[e] = (x[e] + alpha * (double)g[e]) + omega * (double)u;
      const T rn = q - om * y;
      const T kn = u - om * (m - a * n[e]);
      const T wn = y - om * (t[e] - a * v[e]);
      r[e] = rn; k[e] = kn; w[e] = wn;
      const double rhd = (double)rh[e];
      acc[0] += rhd * (double)rn;
      acc[1] += rhd * (double)wn;
      acc[2] += rhd * (double)s[e];
      acc[3] += rhd * (double)z[e];
      acc[4] += (double)rn * (double)rn;
    }
    stc<T, C, NT>(B.r + i, r); stc<T, C, NT>(B.k + i, k); stc<T, C, NT>(B.w + i, w);
    stc<double, C, NT>(B.x + i, x);
    if (FUSE) stc<T, C, NT>(B.v + i, v);
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
static void phaseA_t(Solver& S, bool tr, hipStream_t st) {
  PhaseAArgs<T> a;
  a.k = (const T*)S.vec[V_K]; a.w = (const T*)S.vec[V_W]; a.t = (T*)S.vec[V_T];
  a.r = (const T*)S.vec[V_R]; a.v = (const T*)S.vec[V_V];
  a.g = (T*)S.vec[V_G]; a.s = (T*)S.vec[V_S]; a.l = (T*)S.vec[V_L]; a.z = (T*)S.vec[V_Z];
  a.zsave = (const T*)S.vec[V_TMP];
  a.dinv = (const T*)S.dinv; a.dinv_s = (T)S.dinv_s;
  const int kind = fused_kind(S, tr);
  const StParams<T> P = st_params<T>(S, op_of(S, tr));
  const int64_t nt = S.npad / (kBlock * V16<T>::n);
  const bool ntm = (S.vnt & 1) != 0;
  with_fused_kind<PC>(kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(S.nblk), dim3(kBlock), 0, st, a, P, S.n, S.sc, S.partials, nt);
    };
    if (S.auto_rr) {
      if (ntm) go(k_phaseA<T, PC, true, true, K>); else go(k_phaseA<T, PC, false, true, K>);
    } else {
      if (ntm) go(k_phaseA<T, PC, true, false, K>); else go(k_phaseA<T, PC, false, false, K>);
    }
  });
}

template <typename T, int PC>
static void phaseB_t(Solver& S, bool tr, hipStream_t st) {
  PhaseBArgs<T> a;
  a.x = S.x;
  a.g = (const T*)S.vec[V_G]; a.l = (const T*)S.vec[V_L]; a.s = (const T*)S.vec[V_S];
  a.z = (const T*)S.vec[V_Z]; a.t = (const T*)S.vec[V_T]; a.v = (T*)S.vec[V_V];
  a.rhat = (const T*)S.vec[V_RHAT];
  a.r = (T*)S.vec[V_R]; a.k = (T*)S.vec[V_K]; a.w = (T*)S.vec[V_W];
  a.dinv = (const T*)S.dinv; a.dinv_s = (T)S.dinv_s;
  const int kind = fused_kind(S, tr);
  const StParams<T> P = st_params<T>(S, op_of(S, tr));
  const int64_t nt = S.npad / (kBlock * V16<T>::n);
  const bool ntm = (S.vnt & 2) != 0;
  with_fused_kind<PC>(kind, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(S.nblk), dim3(kBlock), 0, st, a, P, S.n, S.sc, S.partials, nt);
    };
    if (S.auto_rr) {
      if (ntm) go(k_phaseB<T, PC, true, true, K>); else go(k_phaseB<T, PC, false, true, K>);
    } else {
      if (ntm) go(k_phaseB<T, PC, true, false, K>); else go(k_phaseB<T, PC, false, false, K>);
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

void launch_phaseA(Solver& S, bool tr, hipStream_t st) { PBCG_DISPATCH_T_PC(S, phaseA_t, S, tr, st); }
void launch_phaseB(Solver& S, bool tr, hipStream_t st) { PBCG_DISPATCH_T_PC(S, phaseB_t, S, tr, st); }
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
