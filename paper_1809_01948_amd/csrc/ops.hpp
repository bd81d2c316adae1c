// Sparse operators of the library, as row visitors.
//
// Each operator exposes `row(i, vis)`, which calls `vis(a_ij, j)` for the
// stored entries of row i in ascending column order.  The visitor decides
// what is computed (an SPMV with the Jacobi preconditioner fused into the
// input, two products at once for residual replacement, a residual in FP64,
// a gradient ...).  Summing in ascending column order, one rounding per
// multiply and per add (the library is compiled without FMA contraction),
// reproduces a sequential CSR product exactly.
#pragma once

#include "common.hpp"

namespace pbcg {

enum OpKind : int { OP_SELL = 0, OP_ST2D5 = 1, OP_ST3D7 = 2, OP_DIA5 = 3 };

// Sliced ELLPACK with slice height 64 (one wavefront per slice): rows
// [64 s, 64 s + 64) share a width w_s = max row length of the slice; entry j
// of row i sits at sptr[s] + j*64 + (i % 64).  Padding has col = -1.
template <typename T>
struct SellOp {
  const int64_t* __restrict__ sptr;
  const int32_t* __restrict__ col;
  const T* __restrict__ val;
  template <class Vis>
  __device__ __forceinline__ void row(int64_t i, Vis& vis) const {
    const int64_t s = i >> 6;
    const int lane = (int)(i & 63);
    const int64_t off = sptr[s];
    const int w = (int)((sptr[s + 1] - off) >> 6);
    const int32_t* c = col + off + lane;
    const T* a = val + off + lane;
    for (int j = 0; j < w; ++j) {
      const int32_t cj = c[(int64_t)j * kSellC];
      if (cj >= 0) vis(a[(int64_t)j * kSellC], (int64_t)cj);
    }
  }
};

// Constant-coefficient 5-point stencil on an nx x ny grid (p = ix + nx*iy),
// coefficients in ascending column order S, W, C, E, N.
template <typename T>
struct St2d5Op {
  int nx, ny;
  T c[5];
  template <class Vis>
  __device__ __forceinline__ void row(int64_t i, Vis& vis) const {
    const int p = (int)i;
    const int iy = p / nx;
    const int ix = p - iy * nx;
    if (iy > 0) vis(c[0], (int64_t)(p - nx));
    if (ix > 0) vis(c[1], (int64_t)(p - 1));
    vis(c[2], (int64_t)p);
    if (ix < nx - 1) vis(c[3], (int64_t)(p + 1));
    if (iy < ny - 1) vis(c[4], (int64_t)(p + nx));
  }
};

// Constant-coefficient 7-point stencil on nx x ny x nz, coefficients in
// ascending column order D, S, W, C, E, N, U.
template <typename T>
struct St3d7Op {
  int nx, ny, nz;
  T c[7];
  template <class Vis>
  __device__ __forceinline__ void row(int64_t i, Vis& vis) const {
    const int p = (int)i;
    const int nxy = nx * ny;
    const int iz = p / nxy;
    const int rem = p - iz * nxy;
    const int iy = rem / nx;
    const int ix = rem - iy * nx;
    if (iz > 0) vis(c[0], (int64_t)(p - nxy));
    if (iy > 0) vis(c[1], (int64_t)(p - nx));
    if (ix > 0) vis(c[2], (int64_t)(p - 1));
    vis(c[3], (int64_t)p);
    if (ix < nx - 1) vis(c[4], (int64_t)(p + 1));
    if (iy < ny - 1) vis(c[5], (int64_t)(p + nx));
    if (iz < nz - 1) vis(c[6], (int64_t)(p + nxy));
  }
};

// Variable-coefficient five-diagonal matrix on an nx x ny grid: coefficient
// d of row p is dia[d * ld + p], d = S, W, C, E, N.
template <typename T>
struct Dia5Op {
  int nx, ny;
  int64_t ld;
  const T* __restrict__ dia;
  template <class Vis>
  __device__ __forceinline__ void row(int64_t i, Vis& vis) const {
    const int p = (int)i;
    const int iy = p / nx;
    const int ix = p - iy * nx;
    if (iy > 0) vis(dia[i], (int64_t)(p - nx));
    if (ix > 0) vis(dia[ld + i], (int64_t)(p - 1));
    vis(dia[2 * ld + i], (int64_t)p);
    if (ix < nx - 1) vis(dia[3 * ld + i], (int64_t)(p + 1));
    if (iy < ny - 1) vis(dia[4 * ld + i], (int64_t)(p + nx));
  }
};

// ----------------------------------------------------------------------------
// final reductions (one block)
// ----------------------------------------------------------------------------

__device__ __forceinline__ void stop(DevScalars* sc, int status) {
  sc->done = STOPPED;
  sc->status = status;
}

// Runs one FinalMode over the partials written by the previous kernel(s).
// Must be executed by all kBlock threads of exactly one block.
__device__ inline void run_final(int mode, DevScalars* __restrict__ sc,
                                 const double* __restrict__ partials, int nblk, int aux) {
  const bool t0 = threadIdx.x == 0;
  switch (mode) {
    case FIN_INIT: {
      // Algorithm 2 initialisation: rho_0 = (r0, r0), alpha_0 = rho_0 / (r0, w0)
      const double rho = block_sum_slot(partials, SL_RR0, nblk);
      const double rw = block_sum_slot(partials, SL_RW0, nblk);
      const double rr = block_sum_slot(partials, SL_RR, nblk);
      const double bb = block_sum_slot(partials, SL_BB, nblk);
      if (t0) {
        sc->sig[SL_RR0] = rho; sc->sig[SL_RW0] = rw; sc->sig[SL_RR] = rr; sc->sig[SL_BB] = bb;
        sc->rho = rho;
        sc->rn0 = sqrt(rr);
        sc->rn = sc->rn0;
        sc->nb = sqrt(bb);
        sc->beta = 0.0;
        sc->omega = 0.0;
        sc->omega_prev = 0.0;
        sc->iter = 0;
        if (sc->nb == 0.0) stop(sc, ST_CONVERGED);
        else if (sc->rn0 <= sc->tol * sc->nb) stop(sc, ST_CONVERGED);
        else if (!finite(rho) || !finite(rw)) stop(sc, ST_NONFINITE);
        else if (rw == 0.0) stop(sc, ST_BREAKDOWN_RHO);
        else sc->alpha = rho / rw;
      }
      break;
    }
    case FIN_OMEGA:
    case FIN_C_OMEGA: {
      // omega_i = (q_i, y_i) / (y_i, y_i); (y, y) = 0 gives omega = 0
      const double s1 = block_sum_slot(partials, SL_QY, nblk);
      const double s2 = block_sum_slot(partials, SL_YY, nblk);
      if (t0) {
        sc->sig[SL_QY] = s1; sc->sig[SL_YY] = s2;
        sc->n_saved = 0;                       // phase A of this iteration has consumed it
        if (!finite(s1) || !finite(s2)) stop(sc, ST_NONFINITE);
        else sc->omega = (s2 != 0.0) ? s1 / s2 : 0.0;
      }
      break;
    }
    case FIN_BETA:
    case FIN_REDO: {
      // GLRED 2: beta_{i+1} = (alpha_i/omega_i) (r0,r_{i+1})/(r0,r_i),
      // alpha_{i+1} = (r0,r_{i+1}) / ((r0,w_{i+1}) + beta (r0,s_i) - beta omega (r0,z_i))
      const double rho1 = block_sum_slot(partials, SL_RR0, nblk);
      const double rw = block_sum_slot(partials, SL_RW0, nblk);
      const double rs = block_sum_slot(partials, SL_RS0, nblk);
      const double rz = block_sum_slot(partials, SL_RZ0, nblk);
      const double rr = block_sum_slot(partials, SL_RR, nblk);
      if (t0) {
        sc->sig[SL_RR0] = rho1; sc->sig[SL_RW0] = rw; sc->sig[SL_RS0] = rs;
        sc->sig[SL_RZ0] = rz; sc->sig[SL_RR] = rr;
        int its = sc->iter;
        if (mode == FIN_BETA) sc->iter = ++its;
        double* hrow = (sc->history && its >= 1 && its <= sc->hist_len)
                           ? sc->history + 4 * (int64_t)(its - 1) : nullptr;
        if (hrow) { hrow[1] = sc->alpha; hrow[2] = sc->omega; hrow[3] = 0.0; }
        if (!finite(rho1) || !finite(rw) || !finite(rs) || !finite(rz) || !finite(rr)) {
          stop(sc, ST_NONFINITE);
        } else {
          const double rn = sqrt(rr);
          sc->rn = rn;
          if (hrow) hrow[0] = rn;
          if (rn <= sc->tol * sc->nb) {
            sc->done = RECURSIVE_CONVERGED;          // the host confirms with ||b - A x||
          } else if (sc->omega == 0.0) {
            stop(sc, ST_BREAKDOWN_OMEGA);
          } else if (rho1 == 0.0 || sc->rho == 0.0) {
            stop(sc, ST_BREAKDOWN_RHO);
          } else {
            const double beta = ((sc->alpha / sc->omega) * rho1) / sc->rho;
            const double den = (rw + beta * rs) - (beta * sc->omega) * rz;
            if (den == 0.0) {
              stop(sc, ST_BREAKDOWN_RHO);
            } else {
              sc->beta = beta;
              if (hrow) hrow[3] = beta;
              sc->alpha = rho1 / den;
              sc->rho = rho1;
              sc->omega_prev = sc->omega;
              if (its >= sc->maxit) stop(sc, ST_MAXIT);
            }
          }
        }
      }
      break;
    }
    case FIN_TRUE: {
      const double rr = block_sum_slot(partials, SL_RR, nblk);
      if (t0) sc->tr = sqrt(rr);
      break;
    }
    case FIN_GAP: {
      const double rr = block_sum_slot(partials, SL_RR, nblk);
      if (t0) {
        sc->gap = sqrt(rr);
        if (sc->gap_history && sc->gap_idx < sc->gap_len) sc->gap_history[sc->gap_idx] = sc->gap;
        sc->gap_idx += 1;
      }
      break;
    }
    case FIN_C_INIT: {
      // Algorithm 1 initialisation: rho_0 = (r0, r0)
      const double rho = block_sum_slot(partials, SL_RR0, nblk);
      const double rr = block_sum_slot(partials, SL_RR, nblk);
      const double bb = block_sum_slot(partials, SL_BB, nblk);
      if (t0) {
        sc->rho = rho;
        sc->rn0 = sqrt(rr);
        sc->rn = sc->rn0;
        sc->nb = sqrt(bb);
        sc->alpha = sc->beta = sc->omega = sc->omega_prev = 0.0;
        sc->iter = 0;
        if (sc->nb == 0.0) stop(sc, ST_CONVERGED);
        else if (sc->rn0 <= sc->tol * sc->nb) stop(sc, ST_CONVERGED);
        else if (!finite(rho)) stop(sc, ST_NONFINITE);
      }
      break;
    }
    case FIN_C_ALPHA: {
      const double sig = block_sum_slot(partials, SL_RS0, nblk);
      if (t0) {
        sc->sig[SL_RS0] = sig;
        if (!finite(sig)) stop(sc, ST_NONFINITE);
        else if (sig == 0.0) stop(sc, ST_BREAKDOWN_RHO);
        else sc->alpha = sc->rho / sig;
      }
      break;
    }
    case FIN_C_BETA: {
      const double rho1 = block_sum_slot(partials, SL_RR0, nblk);
      const double rr = block_sum_slot(partials, SL_RR, nblk);
      if (t0) {
        sc->sig[SL_RR0] = rho1; sc->sig[SL_RR] = rr;
        const int its = ++sc->iter;
        double* hrow = (sc->history && its <= sc->hist_len)
                           ? sc->history + 4 * (int64_t)(its - 1) : nullptr;
        if (hrow) { hrow[1] = sc->alpha; hrow[2] = sc->omega; hrow[3] = 0.0; }
        if (!finite(rho1) || !finite(rr)) {
          stop(sc, ST_NONFINITE);
        } else {
          const double rn = sqrt(rr);
          sc->rn = rn;
          if (hrow) hrow[0] = rn;
          if (rn <= sc->tol * sc->nb) {
            sc->done = RECURSIVE_CONVERGED;
          } else if (sc->omega == 0.0) {
            stop(sc, ST_BREAKDOWN_OMEGA);
          } else if (rho1 == 0.0) {
            stop(sc, ST_BREAKDOWN_RHO);
          } else {
            sc->beta = ((sc->alpha / sc->omega) * rho1) / sc->rho;
            if (hrow) hrow[3] = sc->beta;
            sc->rho = rho1;
            if (its >= sc->maxit) stop(sc, ST_MAXIT);
          }
        }
      }
      break;
    }
    case FIN_SUM: {
      for (int j = 0; j < aux; ++j) {
        const double v = block_sum_slot(partials, j, nblk);
        if (t0) sc->sums[j] = v;
      }
      break;
    }
    default:
      break;
  }
}

}  // namespace pbcg
