// Operator kernels of pipelined BiCGStab.
//
// Every kernel walks rows in tiles of 256 with the XCD-aware mapping of
// XcdWalk and applies the operator through a row visitor (ops.hpp).
//
// The SPMV kernels carry a global-reduction "final" in their first blocks
// (one block per reduced sum, the last to finish computes the scalars): the
// GLRED of Algorithm 2 is turned into omega_i (or beta_{i+1}, alpha_{i+1})
// while the other blocks compute the SPMV that the reduction is meant to
// hide behind (the PREC + SPMV between "begin global reduction" and "end
// reduction").  The first blocks are dispatched first, so the reduction
// overlaps the whole product.  For structured operators the iteration does
// not use these SPMV kernels (the phase kernels compute the products and
// the GLRED steps; kernels_vec.hip); they serve the initialisation, the
// replacement and operators stored as SELL.

#include <type_traits>

#include "solver.hpp"

namespace pbcg {

// ----------------------------------------------------------------------------
// visitors
// ----------------------------------------------------------------------------

// sum_j a_ij (M^-1 z)_j in the storage precision
template <typename T, int PC>
struct SpmvVis {
  typedef T V;
  const T* __restrict__ z;
  const T* __restrict__ dinv;
  T ds;
  T sum;
  __device__ __forceinline__ V load(int64_t j) const { return prec1<T, PC>(z[j], dinv, ds, j); }
  __device__ __forceinline__ void add(T a, V x) { sum += a * x; }
};

// sum_j a_ij x_j in FP64 (x FP64)
template <typename T>
struct ResVis {
  typedef double V;
  const double* __restrict__ x;
  double sum;
  __device__ __forceinline__ V load(int64_t j) const { return x[j]; }
  __device__ __forceinline__ void add(T a, V v) { sum += (double)a * v; }
};

struct D2 {
  double x, y;
};

// two FP64 products sharing the matrix loads: sum a_ij x_j and sum a_ij y_j
template <typename T, typename X, typename Y>
struct Res2Vis {
  typedef D2 V;
  const X* __restrict__ x;
  const Y* __restrict__ y;
  double sx, sy;
  __device__ __forceinline__ V load(int64_t j) const { return D2{(double)x[j], (double)y[j]}; }
  __device__ __forceinline__ void add(T a, V v) {
    const double ad = (double)a;
    sx += ad * v.x;
    sy += ad * v.y;
  }
};

// classic method: y_i = sum_j a_ij M^-1 (r_j - alpha s_j)
template <typename T, int PC>
struct QVis {
  typedef T V;
  const T* __restrict__ r;
  const T* __restrict__ s;
  const T* __restrict__ dinv;
  T ds, a;
  T sum;
  __device__ __forceinline__ V load(int64_t j) const {
    const T q = r[j] - a * s[j];
    return prec1<T, PC>(q, dinv, ds, j);
  }
  __device__ __forceinline__ void add(T c, V v) { sum += c * v; }
};

// ----------------------------------------------------------------------------
// kernels
// ----------------------------------------------------------------------------

// out = A (M^-1 in); optional partial (r0, out); block 0 runs `fin_mode`.
template <typename T, int PC, class Op>
__global__ __launch_bounds__(kBlock) void k_spmv(Op op, const T* __restrict__ in, T* __restrict__ out,
                                                 const T* __restrict__ dinv, T ds,
                                                 const T* __restrict__ rhat, int64_t n, int64_t ntiles,
                                                 int nwork, DevScalars* __restrict__ sc,
                                                 double* __restrict__ partials, int fin_mode,
                                                 int dot_rhat, int nfin, int npart) {
  if ((int)blockIdx.x < nfin) {
    const int done = sc->done, rr_auto = sc->rr_auto;
    if (fin_mode == FIN_INIT || fin_mode == FIN_REDO || !done)
      distributed_final(fin_mode, sc, partials, npart, nfin, rr_auto);
    return;
  }
  if (sc->done) return;
  const int blk = blockIdx.x - nfin;
  double acc[1] = {0.0};
  for (XcdWalk w(ntiles, blk, nwork); w.t < w.end; w.t += w.step) {
    const int64_t i = w.t * kBlock + threadIdx.x;
    if (i < n) {
      SpmvVis<T, PC> vis{in, dinv, ds, T(0)};
      op.row(i, vis);
      out[i] = vis.sum;
      if (dot_rhat) acc[0] += (double)rhat[i] * (double)vis.sum;
    }
  }
  if (dot_rhat) {
    const int slots[1] = {SL_RW0};
    block_partials<1>(acc, slots, partials, blk);
  }
}

// sum_j a_ij w_j with w the block's column window of M^-1 z, staged in LDS
template <typename T>
struct LdsVis {
  typedef T V;
  const T* win;
  int64_t lo;
  T sum;
  __device__ __forceinline__ V load(int64_t j) const { return win[j - lo]; }
  __device__ __forceinline__ void add(T a, V x) { sum += a * x; }
};

// out = A (M^-1 in) for a sliced-ELL A whose blocks of kLdsRows rows read a
// narrow column window (banded matrices): each block loads its window of
// M^-1 in once, coalesced, into LDS and the gathers of its rows read LDS
// instead of going through the L1 and L2 one line per lane.  The rows are
// summed by the same SellOp::row in the same order as k_spmv: bitwise the
// same products.  Blocks walk the row blocks XCD-aware (consecutive row
// blocks, whose windows overlap, on one XCD's L2).
template <typename T, int PC>
__global__ __launch_bounds__(kLdsRows) void k_spmv_sell_lds(
    SellOp<T> op, const int32_t* __restrict__ win_lo, const int32_t* __restrict__ win_len,
    const T* __restrict__ in, T* __restrict__ out, const T* __restrict__ dinv, T ds, int64_t n,
    int64_t nlb, int nwork, const DevScalars* __restrict__ sc) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* win = (T*)lds_raw;
  if (sc->done) return;
  for (XcdWalk w(nlb, blockIdx.x, nwork); w.t < w.end; w.t += w.step) {
    const int64_t lo = win_lo[w.t];
    const int len = win_len[w.t];
    for (int e = threadIdx.x; e < len; e += kLdsRows)
      win[e] = prec1<T, PC>(in[lo + e], dinv, ds, lo + e);
    __syncthreads();
    const int64_t i = w.t * kLdsRows + threadIdx.x;
    if (i < n) {
      LdsVis<T> vis{win, lo, T(0)};
      op.row(i, vis);
      out[i] = vis.sum;
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// structured SPMV, CH x R consecutive rows per thread
// ----------------------------------------------------------------------------
//
// For the stencil and DIA5 operators with nx a multiple of CH x R (R = 16
// bytes / sizeof(T), CH = 1 or 2 chunks), the rows of a thread lie on one
// grid line, so the centre, S/N (and D/U) neighbours of all its rows are
// aligned 16-byte chunks and the W/E neighbours are the centre chunks
// shifted by one plus one scalar at each end.  Two chunks per thread double
// the bytes each load wave has in flight, which the large grids need to
// approach the HBM bandwidth.  Each row is still summed in ascending column
// order, exactly as the row-per-thread kernel does.

template <typename T, int PC, int KIND, int CH>
__global__ __launch_bounds__(kBlock) void k_spmv_st(StParams<T> P, const T* __restrict__ in,
                                                    T* __restrict__ out, const T* __restrict__ dinv,
                                                    T ds, int64_t n, int64_t ntiles, int nwork,
                                                    DevScalars* __restrict__ sc,
                                                    double* __restrict__ partials, int fin_mode,
                                                    int nblk_partials, int nfin) {
  if ((int)blockIdx.x < nfin) {
    const int done = sc->done, rr_auto = sc->rr_auto;
    if (fin_mode == FIN_INIT || fin_mode == FIN_REDO || !done)
      distributed_final(fin_mode, sc, partials, nblk_partials, nfin, rr_auto);
    return;
  }
  if (sc->done) return;
  constexpr int R = V16<T>::n;
  constexpr int RR = R * CH;           // consecutive rows per thread (CH 16-byte chunks)
  const int blk = blockIdx.x - nfin;
  for (XcdWalk w(ntiles, blk, nwork); w.t < w.end; w.t += w.step) {
    const int64_t p0 = (w.t * kBlock + threadIdx.x) * RR;
    if (p0 >= n) continue;
    const int p = (int)p0;
    T xc[RR], res[RR];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      T t[R];
      load_chunk<T, PC>(in, dinv, ds, p + c * R, t);
#pragma unroll
      for (int e = 0; e < R; ++e) xc[c * R + e] = t[e];
    }
    st_apply<T, PC, KIND, CH>(P, in, dinv, ds, p, xc, res);
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      T t[R];
#pragma unroll
      for (int e = 0; e < R; ++e) t[e] = res[c * R + e];
      st16(out + p + c * R, t);
    }
  }
}

// A GLRED final on its own, spread over one block per reduced slot (the
// automated strategy's 24 sums): block b reduces slot b, the last block to
// finish runs the scalar logic (distributed_final).
__global__ __launch_bounds__(kBlock) void k_fin_dist(int fin_mode, DevScalars* __restrict__ sc,
                                                     const double* __restrict__ partials, int npart) {
  const int done = sc->done, rr_auto = sc->rr_auto;
  if (fin_mode == FIN_INIT || fin_mode == FIN_REDO || !done)
    distributed_final(fin_mode, sc, partials, npart, (int)gridDim.x, rr_auto);
}

// The 3D 7-point product marching through the grid planes: work item
// (zc, c) is segment c of a plane (kBlock * R consecutive rows) in planes
// zc*zlen .. zc*zlen + zlen - 1, visited in order.  A thread keeps the
// chunks of the plane below, the current plane and the plane above in
// registers (each plane's chunk is loaded once, as the next plane up), so
// the +-plane neighbours (a plane apart, 320 KB in FP64) cost no memory
// traffic; the +-line neighbours come from the segments next to it (L1/L2).
// Rows are summed by st_row_sum, so the products equal k_spmv_st's bit for
// bit.  Requires nx a multiple of R.  The first nfin blocks run the final.
template <typename T, int PC>
__global__ __launch_bounds__(kBlock)
void k_spmv_st3m(StParams<T> P, const T* __restrict__ in, T* __restrict__ out,
                 const T* __restrict__ dinv, T ds, int ncol, int nzc, int zlen,
                 DevScalars* __restrict__ sc, double* __restrict__ partials, int fin_mode,
                 int nblk_partials, int nfin) {
  if ((int)blockIdx.x < nfin) {
    const int done = sc->done, rr_auto = sc->rr_auto;
    if (fin_mode == FIN_INIT || fin_mode == FIN_REDO || !done)
      distributed_final(fin_mode, sc, partials, nblk_partials, nfin, rr_auto);
    return;
  }
  if (sc->done) return;
  constexpr int R = V16<T>::n;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int nxy = nx * ny;
  const int blk = blockIdx.x - nfin;
  const int nwork = gridDim.x - nfin;
  const int64_t items = (int64_t)ncol * nzc;
  for (XcdWalk w(items, blk, nwork); w.t < w.end; w.t += w.step) {
    const int zc = (int)(w.t / ncol);
    const int c = (int)(w.t - (int64_t)zc * ncol);
    const int off = c * (kBlock * R) + (int)threadIdx.x * R;
    if (off >= nxy) continue;
    const int iy = off / nx, ix = off - iy * nx;
    const bool hS = iy > 0, hN = iy < ny - 1;
    const bool hW0 = ix > 0, hEl = ix + R < nx;
    const int z0 = zc * zlen;
    const int z1 = z0 + zlen < nz ? z0 + zlen : nz;
    T xd[R], xc[R], xu[R];
    if (z0 > 0) {
      load_chunk<T, PC>(in, dinv, ds, (int64_t)(z0 - 1) * nxy + off, xd);
    } else {
#pragma unroll
      for (int e = 0; e < R; ++e) xd[e] = T(0);           // (no plane below: unused)
    }
    load_chunk<T, PC>(in, dinv, ds, (int64_t)z0 * nxy + off, xc);
    for (int k = z0; k < z1; ++k) {
      const int64_t p = (int64_t)k * nxy + off;
      const bool hD = k > 0, hU = k < nz - 1;
      if (hU) {
        load_chunk<T, PC>(in, dinv, ds, p + nxy, xu);
      } else {
#pragma unroll
        for (int e = 0; e < R; ++e) xu[e] = T(0);         // (no plane above: unused)
      }
      T xs[R], xn[R];
      load_chunk<T, PC>(in, dinv, ds, hS ? p - nx : p, xs);
      load_chunk<T, PC>(in, dinv, ds, hN ? p + nx : p, xn);
      const int64_t jw = hW0 ? p - 1 : p, je = hEl ? p + R : p;
      const T xw0 = prec1<T, PC>(in[jw], dinv, ds, jw);
      const T xeR = prec1<T, PC>(in[je], dinv, ds, je);
      T res[R];
#pragma unroll
      for (int e = 0; e < R; ++e) {
        const T xw = e == 0 ? xw0 : xc[e - 1];
        const T xe = e == R - 1 ? xeR : xc[e + 1];
        const bool vw = e == 0 ? hW0 : true;
        const bool ve = e == R - 1 ? hEl : true;
        res[e] = st_row_sum<T, OP_ST3D7>(P, hD, hS, vw, ve, hN, hU, xd[e], xs[e], xw, xc[e], xe,
                                         xn[e], xu[e], T(0), T(0), T(0), T(0), T(0));
      }
      st16(out + p, res);
#pragma unroll
      for (int e = 0; e < R; ++e) {
        xd[e] = xc[e];
        xc[e] = xu[e];
      }
    }
  }
}

// Algorithm 2 initialisation, first part: r_0 = b - A x_0 (FP64), r0 := r_0,
// k_0 = M^-1 r_0, the iteration -1 vectors g, s, l, z, v set to zero, and the
// partials (r0, r_0), (r_0, r_0), (b, b).
template <typename T, int PC, class Op>
__global__ __launch_bounds__(kBlock) void k_init_res(Op op, const double* __restrict__ x,
                                                     const double* __restrict__ b, T* __restrict__ r,
                                                     T* __restrict__ rhat, T* __restrict__ k,
                                                     T* __restrict__ g, T* __restrict__ s,
                                                     T* __restrict__ l, T* __restrict__ z,
                                                     T* __restrict__ v, const T* __restrict__ dinv,
                                                     T ds, const double* __restrict__ rhat_in,
                                                     int64_t n, int64_t ntiles, int nwork,
                                                     double* __restrict__ partials) {
  const int blk = blockIdx.x;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (XcdWalk w(ntiles, blk, nwork); w.t < w.end; w.t += w.step) {
    const int64_t i = w.t * kBlock + threadIdx.x;
    if (i < n) {
      ResVis<T> vis{x, 0.0};
      op.row(i, vis);
      const T ri = (T)(b[i] - vis.sum);
      const T ki = prec1<T, PC>(ri, dinv, ds, i);
      const T hi = rhat_in ? (T)rhat_in[i] : ri;     // the shadow residual
      r[i] = ri;
      rhat[i] = hi;
      k[i] = ki;
      g[i] = T(0); s[i] = T(0); l[i] = T(0); z[i] = T(0); v[i] = T(0);
      acc[0] += (double)hi * (double)ri;
      acc[1] += (double)ri * (double)ri;
      acc[2] += b[i] * b[i];
      acc[3] += x[i] * x[i];
      acc[4] += (double)ki * (double)ki;
    }
  }
  const int slots[5] = {SL_RR0, SL_RR, SL_BB, SL_X2, SL_K2};
  block_partials<5>(acc, slots, partials, blk);
}

// Every field is loaded before the first test, so that the loads go out
// together (tested one after another they would be dependent round trips).
__device__ __forceinline__ bool rr_due(const DevScalars* __restrict__ sc) {
  const int done = sc->done, rr_auto = sc->rr_auto, rr_next = sc->rr_next;
  const int P = sc->rr_period, iter = sc->iter;
  const double rn = sc->rn, tau = sc->tau, rn0 = sc->rn0;
  if (done) return false;
  if (rr_auto) return rr_next != 0;               // eq:criterion, decided at the last GLRED 2
  if (P <= 0 || ((iter + 1) % P) != 0) return false;
  return rn >= tau * rn0;
}

// A grid smaller than the partial count that the following final reduces
// clears the partials of the blocks it does not have.
template <int NS>
__device__ __forceinline__ void zero_partials(const int (&slot)[NS], double* __restrict__ partials,
                                              int npart) {
  for (int j = blockIdx.x + gridDim.x; j < npart; j += gridDim.x)
    if (threadIdx.x < NS) partials[slot[threadIdx.x] * kMaxPartials + j] = 0.0;
}

// Residual replacement (eq:rr), first half: r = b - A x_{i+1}, k = M^-1 r,
// s = A g_i, l = M^-1 s.  FP64 products; stored results rounded to T.  Also
// the partials of ||x_{i+1}||^2, ||k||^2, ||l||^2 that restart the automated
// replacement bound.
template <typename T, int PC, class Op>
__global__ __launch_bounds__(kBlock) void k_rr1(Op op, const double* __restrict__ x,
                                                const T* __restrict__ g, const double* __restrict__ b,
                                                T* __restrict__ r, T* __restrict__ k, T* __restrict__ s,
                                                T* __restrict__ l, const T* __restrict__ dinv, T ds,
                                                int64_t n, int64_t ntiles, int nwork,
                                                DevScalars* __restrict__ sc,
                                                double* __restrict__ partials, int force,
                                                int npart) {
  if (!force && !rr_due(sc)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->rr_count += 1;
    sc->rr_hit = 1;
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (XcdWalk w(ntiles, blockIdx.x, nwork); w.t < w.end; w.t += w.step) {
    const int64_t i = w.t * kBlock + threadIdx.x;
    if (i < n) {
      Res2Vis<T, double, T> vis{x, g, 0.0, 0.0};
      op.row(i, vis);
      const T ri = (T)(b[i] - vis.sx);
      const T si = (T)vis.sy;
      const T ki = prec1<T, PC>(ri, dinv, ds, i);
      const T li = prec1<T, PC>(si, dinv, ds, i);
      r[i] = ri;
      k[i] = ki;
      s[i] = si;
      l[i] = li;
      acc[0] += x[i] * x[i];
      acc[1] += (double)ki * (double)ki;
      acc[2] += (double)li * (double)li;
      acc[3] += (double)si * (double)si;
    }
  }
  const int slots[4] = {SL_RX2, SL_RK2, SL_RL2, SL_RS2};
  block_partials<4>(acc, slots, partials, blockIdx.x);
  zero_partials<4>(slots, partials, npart);
}

// Residual replacement, second half: w = A k, z = A l (FP64 products), and
// the GLRED 2 partials recomputed from the replaced vectors.  The explicitly
// computed n_i = M^-1 z_i of this iteration is not replaced (only the six
// quantities of eq:rr are), and v_i = A n_i keeps its value; so the
// pre-replacement z_i is kept in `zsave` for the next phase A, which forms
// n_i from it (`save_z` = 0 when an earlier replacement of the same iteration
// has saved it already).  With `keep_n` = 0 (option rr_nv, outside the
// paper) n_i and v_i are refreshed from the replaced z_i instead (k_rr3):
// nothing is saved and the next phase A forms n_i from z_i.  With `pm`, also
// M^-1 w (dinv a vector) for the next product.  Also the partial of ||z||^2
// for the automated bound.
template <typename T, int PC, class Op>
__global__ __launch_bounds__(kBlock) void k_rr2(Op op, const T* __restrict__ k, const T* __restrict__ l,
                                                T* __restrict__ w, T* __restrict__ z,
                                                T* __restrict__ zsave, T* __restrict__ pm,
                                                const T* __restrict__ dinv,
                                                const T* __restrict__ rhat, const T* __restrict__ r,
                                                const T* __restrict__ s, int64_t n, int64_t ntiles,
                                                int nwork, DevScalars* __restrict__ sc,
                                                double* __restrict__ partials, int force,
                                                int npart, int save_z, int keep_n) {
  if (!force && !rr_due(sc)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0 && keep_n) sc->n_saved = 1;
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (XcdWalk wk(ntiles, blockIdx.x, nwork); wk.t < wk.end; wk.t += wk.step) {
    const int64_t i = wk.t * kBlock + threadIdx.x;
    if (i < n) {
      Res2Vis<T, T, T> vis{k, l, 0.0, 0.0};
      op.row(i, vis);
      const T wi = (T)vis.sx;
      const T zi = (T)vis.sy;
      if (save_z && keep_n) zsave[i] = z[i];
      w[i] = wi;
      z[i] = zi;
      if (pm) pm[i] = dinv[i] * wi;
      const double rh = (double)rhat[i], ri = (double)r[i];
      acc[0] += rh * ri;
      acc[1] += rh * (double)wi;
      acc[2] += rh * (double)s[i];
      acc[3] += rh * (double)zi;
      acc[4] += ri * ri;
      acc[5] += (double)zi * (double)zi;
    }
  }
  const int slots[6] = {SL_RR0, SL_RW0, SL_RS0, SL_RZ0, SL_RR, SL_RZ2};
  block_partials<6>(acc, slots, partials, blockIdx.x);
  zero_partials<6>(slots, partials, npart);
}

// Option rr_nv (outside the paper): after a replacement, v_i = A M^-1 z_i
// from the replaced z_i, so that the next iteration's l and z recurrences
// use n_i = M^-1 z_i and v_i = A n_i of the same z_i (the next phase A forms
// n_i from z_i itself).  Predicated like k_rr1 and k_rr2.
template <typename T, int PC, class Op>
__global__ __launch_bounds__(kBlock) void k_rr3(Op op, const T* __restrict__ z, T* __restrict__ v,
                                                const T* __restrict__ dinv, T ds, int64_t n,
                                                int64_t ntiles, int nwork,
                                                const DevScalars* __restrict__ sc, int force) {
  if (!force && !rr_due(sc)) return;
  for (XcdWalk wk(ntiles, blockIdx.x, nwork); wk.t < wk.end; wk.t += wk.step) {
    const int64_t i = wk.t * kBlock + threadIdx.x;
    if (i < n) {
      SpmvVis<T, PC> vis{z, dinv, ds, T(0)};
      op.row(i, vis);
      v[i] = vis.sum;
    }
  }
}

// partial of ||b - A x||^2 (FP64)
template <typename T, class Op>
__global__ __launch_bounds__(kBlock) void k_true_res(Op op, const double* __restrict__ x,
                                                     const double* __restrict__ b, int64_t n,
                                                     int64_t ntiles, int nwork,
                                                     double* __restrict__ partials) {
  double acc[1] = {0.0};
  for (XcdWalk w(ntiles, blockIdx.x, nwork); w.t < w.end; w.t += w.step) {
    const int64_t i = w.t * kBlock + threadIdx.x;
    if (i < n) {
      ResVis<T> vis{x, 0.0};
      op.row(i, vis);
      const double ri = b[i] - vis.sum;
      acc[0] += ri * ri;
    }
  }
  const int slots[1] = {SL_RR};
  block_partials<1>(acc, slots, partials, blockIdx.x);
}

// partial of ||(b - A x) - r||^2, the residual gap of eq:res_gap
template <typename T, class Op>
__global__ __launch_bounds__(kBlock) void k_gap(Op op, const double* __restrict__ x,
                                                const double* __restrict__ b, const T* __restrict__ r,
                                                int64_t n, int64_t ntiles, int nwork,
                                                DevScalars* __restrict__ sc,
                                                double* __restrict__ partials, int force) {
  if (sc->done && !force) return;
  double acc[1] = {0.0};
  for (XcdWalk w(ntiles, blockIdx.x, nwork); w.t < w.end; w.t += w.step) {
    const int64_t i = w.t * kBlock + threadIdx.x;
    if (i < n) {
      ResVis<T> vis{x, 0.0};
      op.row(i, vis);
      const double gi = (b[i] - vis.sum) - (double)r[i];
      acc[0] += gi * gi;
    }
  }
  const int slots[1] = {SL_RR};
  block_partials<1>(acc, slots, partials, blockIdx.x);
}

// Algorithm 1 initialisation: r_0 = b - A x_0, r0 := r_0, p_0 := r_0
template <typename T, class Op>
__global__ __launch_bounds__(kBlock) void k_cl_init(Op op, const double* __restrict__ x,
                                                    const double* __restrict__ b, T* __restrict__ r,
                                                    T* __restrict__ rhat, T* __restrict__ p,
                                                    const double* __restrict__ rhat_in, int64_t n,
                                                    int64_t ntiles, int nwork,
                                                    double* __restrict__ partials) {
  double acc[3] = {0.0, 0.0, 0.0};
  for (XcdWalk w(ntiles, blockIdx.x, nwork); w.t < w.end; w.t += w.step) {
    const int64_t i = w.t * kBlock + threadIdx.x;
    if (i < n) {
      ResVis<T> vis{x, 0.0};
      op.row(i, vis);
      const T ri = (T)(b[i] - vis.sum);
      const T hi = rhat_in ? (T)rhat_in[i] : ri;     // the shadow residual
      r[i] = ri; rhat[i] = hi; p[i] = ri;
      acc[0] += (double)hi * (double)ri;
      acc[1] += (double)ri * (double)ri;
      acc[2] += b[i] * b[i];
    }
  }
  const int slots[3] = {SL_RR0, SL_RR, SL_BB};
  block_partials<3>(acc, slots, partials, blockIdx.x);
}

// Algorithm 1: s_i = A M^-1 p_i and the partial (r0, s_i)
template <typename T, int PC, class Op>
__global__ __launch_bounds__(kBlock) void k_cl_spmv_s(Op op, const T* __restrict__ p, T* __restrict__ s,
                                                      const T* __restrict__ rhat,
                                                      const T* __restrict__ dinv, T ds, int64_t n,
                                                      int64_t ntiles, int nwork,
                                                      const DevScalars* __restrict__ sc,
                                                      double* __restrict__ partials) {
  if (sc->done) return;
  double acc[1] = {0.0};
  for (XcdWalk w(ntiles, blockIdx.x, nwork); w.t < w.end; w.t += w.step) {
    const int64_t i = w.t * kBlock + threadIdx.x;
    if (i < n) {
      SpmvVis<T, PC> vis{p, dinv, ds, T(0)};
      op.row(i, vis);
      s[i] = vis.sum;
      acc[0] += (double)rhat[i] * (double)vis.sum;
    }
  }
  const int slots[1] = {SL_RS0};
  block_partials<1>(acc, slots, partials, blockIdx.x);
}

// Algorithm 1: y_i = A M^-1 q_i with q = r - alpha s formed on the fly, and
// the partials (q_i, y_i), (y_i, y_i)
template <typename T, int PC, class Op>
__global__ __launch_bounds__(kBlock) void k_cl_spmv_y(Op op, const T* __restrict__ r,
                                                      const T* __restrict__ s, T* __restrict__ y,
                                                      const T* __restrict__ dinv, T ds, int64_t n,
                                                      int64_t ntiles, int nwork,
                                                      const DevScalars* __restrict__ sc,
                                                      double* __restrict__ partials) {
  const int done = sc->done;
  const double alpha = sc->alpha;
  if (done) return;
  const T a = (T)alpha;
  double acc[2] = {0.0, 0.0};
  for (XcdWalk w(ntiles, blockIdx.x, nwork); w.t < w.end; w.t += w.step) {
    const int64_t i = w.t * kBlock + threadIdx.x;
    if (i < n) {
      QVis<T, PC> vis{r, s, dinv, ds, a, T(0)};
      op.row(i, vis);
      y[i] = vis.sum;
      const T qi = r[i] - a * s[i];
      acc[0] += (double)qi * (double)vis.sum;
      acc[1] += (double)vis.sum * (double)vis.sum;
    }
  }
  const int slots[2] = {SL_QY, SL_YY};
  block_partials<2>(acc, slots, partials, blockIdx.x);
}

// y = A x with FP64 accumulation (user buffers of length n)
template <typename T, class Op>
__global__ __launch_bounds__(kBlock) void k_apply(Op op, const double* __restrict__ x,
                                                  double* __restrict__ y, int64_t n, int64_t ntiles,
                                                  int nwork) {
  for (XcdWalk w(ntiles, blockIdx.x, nwork); w.t < w.end; w.t += w.step) {
    const int64_t i = w.t * kBlock + threadIdx.x;
    if (i < n) {
      ResVis<T> vis{x, 0.0};
      op.row(i, vis);
      y[i] = vis.sum;
    }
  }
}

// dL/da_ij = -lambda_i x_j on the CSR pattern (stored order)
__global__ __launch_bounds__(kBlock) void k_grad_csr(const int32_t* __restrict__ rowptr,
                                                     const int32_t* __restrict__ col,
                                                     const double* __restrict__ lam,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ grad, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const double li = lam[i];
    for (int32_t kk = rowptr[i]; kk < rowptr[i + 1]; ++kk) grad[kk] = -li * x[col[kk]];
  }
}

// DIA5 pattern: grad[d * n + p] = -lambda_p x_{p + off_d} (0 where the entry does not exist)
__global__ __launch_bounds__(kBlock) void k_grad_dia5(int nx, int ny, const double* __restrict__ lam,
                                                      const double* __restrict__ x,
                                                      double* __restrict__ grad, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    const int p = (int)i;
    const int iy = p / nx, ix = p - iy * nx;
    const double li = -lam[i];
    grad[i] = iy > 0 ? li * x[p - nx] : 0.0;
    grad[n + i] = ix > 0 ? li * x[p - 1] : 0.0;
    grad[2 * n + i] = li * x[p];
    grad[3 * n + i] = ix < nx - 1 ? li * x[p + 1] : 0.0;
    grad[4 * n + i] = iy < ny - 1 ? li * x[p + nx] : 0.0;
  }
}

// constant stencil: dL/dc_d = sum_p -lambda_p x_{p + off_d} over existing entries
template <int KIND>
__global__ __launch_bounds__(kBlock) void k_grad_st(int nx, int ny, int nz,
                                                    const double* __restrict__ lam,
                                                    const double* __restrict__ x, int64_t n,
                                                    int64_t ntiles, int nwork,
                                                    double* __restrict__ partials) {
  constexpr int ND = KIND == OP_ST2D5 ? 5 : 7;
  double acc[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) acc[d] = 0.0;
  for (XcdWalk w(ntiles, blockIdx.x, nwork); w.t < w.end; w.t += w.step) {
    const int64_t i = w.t * kBlock + threadIdx.x;
    if (i < n) {
      const int p = (int)i;
      const double li = -lam[i];
      if (KIND == OP_ST2D5) {
        const int iy = p / nx, ix = p - iy * nx;
        if (iy > 0) acc[0] += li * x[p - nx];
        if (ix > 0) acc[1] += li * x[p - 1];
        acc[2] += li * x[p];
        if (ix < nx - 1) acc[3] += li * x[p + 1];
        if (iy < ny - 1) acc[4] += li * x[p + nx];
      } else {
        const int nxy = nx * ny;
        const int iz = p / nxy, rem = p - iz * nxy, iy = rem / nx, ix = rem - iy * nx;
        if (iz > 0) acc[0] += li * x[p - nxy];
        if (iy > 0) acc[1] += li * x[p - nx];
        if (ix > 0) acc[2] += li * x[p - 1];
        acc[3] += li * x[p];
        if (ix < nx - 1) acc[4] += li * x[p + 1];
        if (iy < ny - 1) acc[5] += li * x[p + nx];
        if (iz < nz - 1) acc[6] += li * x[p + nxy];
      }
    }
  }
  int slots[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) slots[d] = d;
  block_partials<ND>(acc, slots, partials, blockIdx.x);
}

// value update of a SELL operator from CSR-ordered values, and Jacobi diagonal
template <typename T>
__global__ void k_update_sell(const double* __restrict__ val, int64_t nnz,
                              const int64_t* __restrict__ pos, T* __restrict__ sv) {
  for (int64_t kk = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; kk < nnz;
       kk += (int64_t)gridDim.x * blockDim.x)
    sv[pos[kk]] = (T)val[kk];
}

template <typename T>
__global__ void k_update_dinv(const double* __restrict__ val, const int64_t* __restrict__ diagpos,
                              T* __restrict__ dinv, int64_t n, int32_t* __restrict__ bad) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t dp = diagpos[i];
    const T d = dp >= 0 ? (T)val[dp] : T(0);
    if (d == T(0)) {
      *bad = 1;
      dinv[i] = T(0);
    } else {
      dinv[i] = T(1) / d;
    }
  }
}

// DIA5 coefficients of -div(kappa grad u) + (cx, cy).grad u (h^2-scaled),
// face value = mean of the two node values, own value on a boundary face;
// also the transposed DIA5 and the Jacobi diagonal.
template <typename T>
__global__ void k_kappa_assemble(const double* __restrict__ kap, int nx, int ny, double cx,
                                 double cy, double h, T* __restrict__ dia, T* __restrict__ diaT,
                                 int64_t ld, T* __restrict__ dinv, int32_t* __restrict__ bad) {
  const int64_t n = (int64_t)nx * ny;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)i;
    const int iy = p / nx, ix = p - iy * nx;
    const double kp = kap[p];
    const double ke = ix < nx - 1 ? 0.5 * (kp + kap[p + 1]) : kp;
    const double kw = ix > 0 ? 0.5 * (kp + kap[p - 1]) : kp;
    const double kn = iy < ny - 1 ? 0.5 * (kp + kap[p + nx]) : kp;
    const double ks = iy > 0 ? 0.5 * (kp + kap[p - nx]) : kp;
    const double C = ((ke + kw) + kn) + ks;
    const double E = ix < nx - 1 ? -ke + cx * h / 2.0 : 0.0;
    const double W = ix > 0 ? -kw - cx * h / 2.0 : 0.0;
    const double N = iy < ny - 1 ? -kn + cy * h / 2.0 : 0.0;
    const double S = iy > 0 ? -ks - cy * h / 2.0 : 0.0;
    dia[i] = (T)S; dia[ld + i] = (T)W; dia[2 * ld + i] = (T)C; dia[3 * ld + i] = (T)E;
    dia[4 * ld + i] = (T)N;
    const T Ct = (T)C;
    if (Ct == T(0)) { *bad = 1; dinv[i] = T(0); } else { dinv[i] = T(1) / Ct; }
  }
  (void)diaT;
}

// transposed DIA5: A^T(p, p-nx) = A(p-nx, p) = N of row p-nx, etc.
template <typename T>
__global__ void k_dia5_transpose(const T* __restrict__ dia, T* __restrict__ diaT, int nx, int ny,
                                 int64_t ld) {
  const int64_t n = (int64_t)nx * ny;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)i;
    const int iy = p / nx, ix = p - iy * nx;
    diaT[i] = iy > 0 ? dia[4 * ld + (p - nx)] : T(0);
    diaT[ld + i] = ix > 0 ? dia[3 * ld + (p - 1)] : T(0);
    diaT[2 * ld + i] = dia[2 * ld + i];
    diaT[3 * ld + i] = ix < nx - 1 ? dia[ld + (p + 1)] : T(0);
    diaT[4 * ld + i] = iy < ny - 1 ? dia[(p + nx)] : T(0);
  }
}

// dL/dkappa from the face gradients -(lam_p - lam_q)(x_p - x_q) (interior
// faces, half to each node) and -lam_p x_p (boundary faces)
__global__ void k_kappa_grad(const double* __restrict__ lam, const double* __restrict__ x, int nx,
                             int ny, double* __restrict__ gk) {
  const int64_t n = (int64_t)nx * ny;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)i;
    const int iy = p / nx, ix = p - iy * nx;
    const double lp = lam[p], xp = x[p];
    double g = 0.0;
    if (ix < nx - 1) g += 0.5 * (-(lp - lam[p + 1]) * (xp - x[p + 1]));
    if (ix > 0) g += 0.5 * (-(lam[p - 1] - lp) * (x[p - 1] - xp));
    if (iy < ny - 1) g += 0.5 * (-(lp - lam[p + nx]) * (xp - x[p + nx]));
    if (iy > 0) g += 0.5 * (-(lam[p - nx] - lp) * (x[p - nx] - xp));
    const double own = -lp * xp;
    if (ix == 0) g += own;
    if (ix == nx - 1) g += own;
    if (iy == 0) g += own;
    if (iy == ny - 1) g += own;
    gk[i] = g;
  }
}

// ----------------------------------------------------------------------------
// dispatch
// ----------------------------------------------------------------------------

const OpData& op_of(Solver& S, bool transpose) { return transpose ? S.AT : S.A; }

template <typename T, class F>
static void with_op_t(Solver& S, const OpData& o, bool use_pc, F& f) {
  switch (o.kind) {
    case OP_SELL: {
      SellOp<T> op{o.sptr, o.col, (const T*)o.val};
      if (use_pc && S.pc == PC_VECTOR) f.template operator()<T, PC_VECTOR>(op);
      else f.template operator()<T, PC_NONE>(op);
      break;
    }
    case OP_ST2D5: {
      St2d5Op<T> op;
      op.nx = o.dims[0]; op.ny = o.dims[1];
      for (int d = 0; d < 5; ++d) op.c[d] = sizeof(T) == 8 ? (T)o.c64[d] : (T)o.c32[d];
      if (use_pc && S.pc == PC_SCALAR) f.template operator()<T, PC_SCALAR>(op);
      else f.template operator()<T, PC_NONE>(op);
      break;
    }
    case OP_ST3D7: {
      St3d7Op<T> op;
      op.nx = o.dims[0]; op.ny = o.dims[1]; op.nz = o.dims[2];
      for (int d = 0; d < 7; ++d) op.c[d] = sizeof(T) == 8 ? (T)o.c64[d] : (T)o.c32[d];
      if (use_pc && S.pc == PC_SCALAR) f.template operator()<T, PC_SCALAR>(op);
      else f.template operator()<T, PC_NONE>(op);
      break;
    }
    case OP_DIA5: {
      Dia5Op<T> op;
      op.nx = o.dims[0]; op.ny = o.dims[1]; op.ld = S.npad; op.dia = (const T*)o.dia;
      if (use_pc && S.pc == PC_VECTOR) f.template operator()<T, PC_VECTOR>(op);
      else f.template operator()<T, PC_NONE>(op);
      break;
    }
  }
}

template <class F>
static void with_op(Solver& S, bool tr, bool use_pc, F&& f) {
  const OpData& o = op_of(S, tr);
  if (S.precision == 0) with_op_t<double>(S, o, use_pc, f);
  else with_op_t<float>(S, o, use_pc, f);
}

#define PBCG_GRID_OP dim3(S.nblk), dim3(kBlock), 0, st

// Grid of the replacement kernels.  With the automated criterion they are
// launched every iteration and usually exit at once (the decision is made
// on the device), so a quarter of the usual grid keeps the empty launches
// cheap; the partials of the missing blocks are cleared by the kernels.
static int rr_grid(const Solver& S) {
  const int g = S.auto_rr ? S.nblk / 4 : S.nblk;
  return g < kXcds ? kXcds : (g / kXcds) * kXcds;
}

// blocks that run a fused final at the head of an SpMV grid: one per slot
static int fin_blocks(const Solver& S, int fin_mode) {
  return fin_mode == FIN_NONE ? 0 : fin_slot_count(fin_mode, S.auto_rr ? 1 : 0);
}

template <typename T>
static bool spmv_structured(Solver& S, const OpData& o, const void* in, void* out, int fin_mode,
                            hipStream_t st) {
  constexpr int R = V16<T>::n;
  if (o.kind == OP_SELL || o.dims[0] % R != 0) return false;
  const int nwork = S.nspmv;
  if (o.kind == OP_ST3D7 && S.march3d) {
    // plane-marching 3D product; z-chunks long enough that the work items
    // (segments x z-chunks) about fill the grid once
    const StParams<T> P = st_params<T>(S, o);
    const int64_t nxy = (int64_t)o.dims[0] * o.dims[1];
    const int seg = kBlock * R;
    const int ncol = (int)((nxy + seg - 1) / seg);
    const int nz = o.dims[2];
    int zlen = (int)std::max<int64_t>(1, ((int64_t)ncol * nz + nwork - 1) / nwork);
    if (S.march_zlen > 0) zlen = std::min(S.march_zlen, nz);
    const int nzc = (nz + zlen - 1) / zlen;
    const int nfin = fin_blocks(S, fin_mode);
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(nwork + nfin), dim3(kBlock), 0, st, P, (const T*)in, (T*)out,
                         (const T*)S.dinv, (T)S.dinv_s, ncol, nzc, zlen, S.sc, S.partials,
                         fin_mode, S.nblk, nfin);
    };
    if (S.pc != PC_NONE) go(k_spmv_st3m<T, PC_SCALAR>);
    else go(k_spmv_st3m<T, PC_NONE>);
    return true;
  }
  // two 16-byte chunks per thread (twice the bytes in flight per load wave)
  // when grid lines allow it and the grid still has two tiles per block
  const bool two = o.dims[0] % (2 * R) == 0 &&
                   S.n / ((int64_t)kBlock * 2 * R) >= 2 * (int64_t)nwork;
  const StParams<T> P = st_params<T>(S, o);
  const int64_t rows = (int64_t)kBlock * R * (two ? 2 : 1);
  const int64_t ntiles = (S.n + rows - 1) / rows;
  const int nfin = fin_blocks(S, fin_mode);
  auto go = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(nwork + nfin), dim3(kBlock), 0, st, P, (const T*)in, (T*)out,
                       (const T*)S.dinv, (T)S.dinv_s, S.n, ntiles, nwork, S.sc, S.partials,
                       fin_mode, S.nblk, nfin);
  };
  const bool pc = S.pc != PC_NONE;
  auto pick = [&](auto ch) {
    constexpr int CH = decltype(ch)::value;
    switch (o.kind) {
      case OP_ST2D5:
        if (pc) go(k_spmv_st<T, PC_SCALAR, OP_ST2D5, CH>); else go(k_spmv_st<T, PC_NONE, OP_ST2D5, CH>);
        break;
      case OP_ST3D7:
        if (pc) go(k_spmv_st<T, PC_SCALAR, OP_ST3D7, CH>); else go(k_spmv_st<T, PC_NONE, OP_ST3D7, CH>);
        break;
      case OP_DIA5:
        if (pc) go(k_spmv_st<T, PC_VECTOR, OP_DIA5, CH>); else go(k_spmv_st<T, PC_NONE, OP_DIA5, CH>);
        break;
    }
  };
  if (two) pick(std::integral_constant<int, 2>{});
  else pick(std::integral_constant<int, 1>{});
  return true;
}

// Measured on MI355X: computing the products inside the phase kernels pays
// for 2D grids (constant stencils, DIA5) in both precisions and for 3D grids
// with FP32 storage (200^3: 182 against 197 us per iteration); with FP64
// storage on 3D grids the fused phase kernels re-read the stencil input from
// HBM (plane neighbours 320 KB apart fall out of the L2 under the other
// streams) and the separate SPMVs are faster (356 against 366 us).
int fused_kind(Solver& S, bool tr) {
  if (!S.fuse || !S.spmv_tiled) return 0;
  const OpData& o = op_of(S, tr);
  const int R = (int)(16 / S.tsize);
  if (o.kind == OP_SELL || o.dims[0] % R != 0) return 0;
  if (o.kind == OP_ST3D7 && S.precision == 0) return 0;
  if ((o.kind == OP_ST2D5 || o.kind == OP_ST3D7) && S.pc == PC_VECTOR) return 0;
  if (o.kind == OP_DIA5 && S.pc == PC_SCALAR) return 0;
  return o.kind;
}

// Used with FP32 storage only (200^3: 172.2 -> 171.4 us per iteration, the
// products fused with the planes in registers); in FP64, where the 3D products
// are separate kernels, the march made the phase kernels slower (351 -> 357
// us), and fusing the FP64 products with it slower still (365 us; row order
// fused: 349 us, no gain over the separate products).
int phase_march_planes(Solver& S, bool tr) {
  if (!S.march_phase || S.precision == 0) return 0;
  const OpData& o = op_of(S, tr);
  const int C = (int)(16 / S.tsize);
  if (o.kind != OP_ST3D7 || o.dims[0] % C != 0) return 0;
  const int64_t nxy = (int64_t)o.dims[0] * o.dims[1];
  const int64_t seg = (int64_t)kBlock * C;
  const int64_t ncol = (nxy + seg - 1) / seg;
  const int nz = o.dims[2];
  const int64_t bpx = std::max(1, S.nblk / kXcds);        // blocks per XCD
  // the count (up to 8) that minimises a block's largest number of tiles; the
  // largest such count (most planes visited in order)
  int best = 1;
  int64_t best_max = INT64_MAX;
  for (int mz = 1; mz <= 8 && mz <= nz; ++mz) {
    const int64_t items = ncol * ((nz + mz - 1) / mz);
    const int64_t per_xcd = (items + kXcds - 1) / kXcds;
    const int64_t most = (per_xcd + bpx - 1) / bpx * mz;
    if (most <= best_max) {
      best_max = most;
      best = mz;
    }
  }
  return best;
}

void launch_fin(Solver& S, int fin_mode, hipStream_t st) {
  // up to 8 sums: one block loads them all in one round trip; more (the
  // automated strategy's 24): one block per sum
  const int nfin = fin_blocks(S, fin_mode);
  if (nfin <= 8) {
    launch_final(S, fin_mode, 0, st);
    return;
  }
  hipLaunchKernelGGL(k_fin_dist, dim3(nfin), dim3(kBlock), 0, st, fin_mode, S.sc, S.partials,
                     S.nblk);
}

bool pre_multiplied(Solver& S, bool tr) {
  return S.premult && S.pc == PC_VECTOR && op_of(S, tr).kind == OP_SELL &&
         fused_kind(S, tr) == 0;
}

bool sell_lds_ok(const Solver& S, const OpData& o) {
  return S.sell_lds && o.kind == OP_SELL && o.win_lo && o.win_max > 0 &&
         (int64_t)o.win_max * (int64_t)S.tsize <= S.lds_cap;
}

// The LDS-window product; the GLRED final (if any) runs first as its own
// kernel (the same reduction tree, so the same bits).
static void launch_spmv_lds(Solver& S, bool tr, const void* in, void* out, int fin_mode,
                            hipStream_t st, bool pre) {
  if (fin_mode != FIN_NONE) launch_fin(S, fin_mode, st);
  const OpData& o = op_of(S, tr);
  const size_t shmem = (size_t)o.win_max * S.tsize;
  // one block per CU when the window takes more than half a block's LDS,
  // else two (2e6 x 27 banded matrix, 88 KB FP64 windows: 256 blocks 124 us,
  // 512 126 us; 44 KB FP32 windows: 256 blocks 83 us, 512 78 us)
  const int64_t per_cu = shmem * 2 > (size_t)S.lds_cap ? 1 : 2;
  const int64_t nw = std::min<int64_t>(o.nlb, S.lds_blocks > 0 ? S.lds_blocks : 256 * per_cu);
  const int nwork = (int)std::max<int64_t>(kXcds, nw / kXcds * kXcds);
  with_op(S, tr, !pre, [&]<typename T, int PC, class Op>(const Op& op) {
    if constexpr (std::is_same_v<Op, SellOp<T>>) {
      // (if the attribute is refused, the launch below fails and the
      // caller's launch check reports it)
      static bool attr = false;
      if (!attr)
        attr = hipFuncSetAttribute((const void*)k_spmv_sell_lds<T, PC>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)S.lds_cap) == hipSuccess;
      hipLaunchKernelGGL((k_spmv_sell_lds<T, PC>), dim3(nwork), dim3(kLdsRows), shmem, st, op,
                         o.win_lo, o.win_len, (const T*)in, (T*)out, (const T*)S.dinv,
                         (T)S.dinv_s, S.n, o.nlb, nwork, S.sc);
    }
  });
}

void launch_iter_spmv(Solver& S, bool tr, int in_vec, int out_vec, int fin_mode, hipStream_t st) {
  if (sell_lds_ok(S, op_of(S, tr))) {
    const bool pre = pre_multiplied(S, tr);
    launch_spmv_lds(S, tr, pre ? S.vec[V_PM] : S.vec[in_vec], S.vec[out_vec], fin_mode, st, pre);
    return;
  }
  if (pre_multiplied(S, tr))
    launch_spmv(S, tr, S.vec[V_PM], S.vec[out_vec], fin_mode, false, st, true);
  else
    launch_spmv(S, tr, S.vec[in_vec], S.vec[out_vec], fin_mode, false, st);
}

void launch_spmv(Solver& S, bool tr, const void* in, void* out, int fin_mode, bool dot_rhat,
                 hipStream_t st, bool pre) {
  if (!dot_rhat && S.spmv_tiled && !pre) {
    const OpData& o = op_of(S, tr);
    const bool done = S.precision == 0 ? spmv_structured<double>(S, o, in, out, fin_mode, st)
                                       : spmv_structured<float>(S, o, in, out, fin_mode, st);
    if (done) return;
  }
  const int nfin = fin_blocks(S, fin_mode);
  // the (r0, out) partials are indexed by work block and reduced over nblk
  const int nwork = dot_rhat ? S.nblk : S.nspmv;
  with_op(S, tr, !pre, [&]<typename T, int PC, class Op>(const Op& op) {
    hipLaunchKernelGGL((k_spmv<T, PC, Op>), dim3(nwork + nfin), dim3(kBlock), 0, st, op,
                       (const T*)in, (T*)out, (const T*)S.dinv, (T)S.dinv_s,
                       (const T*)S.vec[V_RHAT], S.n, S.rtiles, nwork, S.sc, S.partials, fin_mode,
                       dot_rhat ? 1 : 0, nfin, S.nblk);
  });
}

void launch_init_res(Solver& S, bool tr, hipStream_t st) {
  with_op(S, tr, true, [&]<typename T, int PC, class Op>(const Op& op) {
    hipLaunchKernelGGL((k_init_res<T, PC, Op>), PBCG_GRID_OP, op, (const double*)S.x,
                       (const double*)S.b, (T*)S.vec[V_R], (T*)S.vec[V_RHAT], (T*)S.vec[V_K],
                       (T*)S.vec[V_G], (T*)S.vec[V_S], (T*)S.vec[V_L], (T*)S.vec[V_Z],
                       (T*)S.vec[V_V], (const T*)S.dinv, (T)S.dinv_s, S.rhat_in, S.n, S.rtiles,
                       S.nblk, S.partials);
  });
}

void launch_rr1(Solver& S, bool tr, bool force, hipStream_t st) {
  with_op(S, tr, true, [&]<typename T, int PC, class Op>(const Op& op) {
    const int g = rr_grid(S);
    hipLaunchKernelGGL((k_rr1<T, PC, Op>), dim3(g), dim3(kBlock), 0, st, op, (const double*)S.x,
                       (const T*)S.vec[V_G], (const double*)S.b, (T*)S.vec[V_R], (T*)S.vec[V_K],
                       (T*)S.vec[V_S], (T*)S.vec[V_L], (const T*)S.dinv, (T)S.dinv_s, S.n,
                       S.rtiles, g, S.sc, S.partials, force ? 1 : 0, S.nblk);
  });
}

void launch_rr2(Solver& S, bool tr, bool force, hipStream_t st, bool save_z, bool keep_n) {
  with_op(S, tr, false, [&]<typename T, int PC, class Op>(const Op& op) {
    const int g = rr_grid(S);
    hipLaunchKernelGGL((k_rr2<T, PC, Op>), dim3(g), dim3(kBlock), 0, st, op, (const T*)S.vec[V_K],
                       (const T*)S.vec[V_L], (T*)S.vec[V_W], (T*)S.vec[V_Z], (T*)S.vec[V_TMP],
                       pre_multiplied(S, tr) ? (T*)S.vec[V_PM] : (T*)nullptr,
                       (const T*)S.dinv, (const T*)S.vec[V_RHAT], (const T*)S.vec[V_R], (const T*)S.vec[V_S], S.n,
                       S.rtiles, g, S.sc, S.partials, force ? 1 : 0, S.nblk, save_z ? 1 : 0,
                       keep_n ? 1 : 0);
  });
}

void launch_rr3(Solver& S, bool tr, bool force, hipStream_t st) {
  with_op(S, tr, true, [&]<typename T, int PC, class Op>(const Op& op) {
    const int g = rr_grid(S);
    hipLaunchKernelGGL((k_rr3<T, PC, Op>), dim3(g), dim3(kBlock), 0, st, op, (const T*)S.vec[V_Z],
                       (T*)S.vec[V_V], (const T*)S.dinv, (T)S.dinv_s, S.n, S.rtiles, g, S.sc,
                       force ? 1 : 0);
  });
}

void launch_true_res(Solver& S, bool tr, hipStream_t st) {
  with_op(S, tr, false, [&]<typename T, int PC, class Op>(const Op& op) {
    hipLaunchKernelGGL((k_true_res<T, Op>), PBCG_GRID_OP, op, (const double*)S.x,
                       (const double*)S.b, S.n, S.rtiles, S.nblk, S.partials);
  });
}

void launch_gap(Solver& S, bool tr, hipStream_t st, bool force) {
  with_op(S, tr, false, [&]<typename T, int PC, class Op>(const Op& op) {
    hipLaunchKernelGGL((k_gap<T, Op>), PBCG_GRID_OP, op, (const double*)S.x, (const double*)S.b,
                       (const T*)S.vec[V_R], S.n, S.rtiles, S.nblk, S.sc, S.partials,
                       force ? 1 : 0);
  });
}

void launch_cl_init(Solver& S, bool tr, hipStream_t st) {
  with_op(S, tr, false, [&]<typename T, int PC, class Op>(const Op& op) {
    hipLaunchKernelGGL((k_cl_init<T, Op>), PBCG_GRID_OP, op, (const double*)S.x,
                       (const double*)S.b, (T*)S.vec[V_R], (T*)S.vec[V_RHAT], (T*)S.vec[V_G],
                       S.rhat_in, S.n, S.rtiles, S.nblk, S.partials);
  });
}

void launch_cl_spmv_s(Solver& S, bool tr, hipStream_t st) {
  with_op(S, tr, true, [&]<typename T, int PC, class Op>(const Op& op) {
    hipLaunchKernelGGL((k_cl_spmv_s<T, PC, Op>), PBCG_GRID_OP, op, (const T*)S.vec[V_G],
                       (T*)S.vec[V_S], (const T*)S.vec[V_RHAT], (const T*)S.dinv, (T)S.dinv_s,
                       S.n, S.rtiles, S.nblk, S.sc, S.partials);
  });
}

void launch_cl_spmv_y(Solver& S, bool tr, hipStream_t st) {
  with_op(S, tr, true, [&]<typename T, int PC, class Op>(const Op& op) {
    hipLaunchKernelGGL((k_cl_spmv_y<T, PC, Op>), PBCG_GRID_OP, op, (const T*)S.vec[V_R],
                       (const T*)S.vec[V_S], (T*)S.vec[V_V], (const T*)S.dinv, (T)S.dinv_s, S.n,
                       S.rtiles, S.nblk, S.sc, S.partials);
  });
}

void launch_apply(Solver& S, bool tr, const double* x, double* y, hipStream_t st) {
  with_op(S, tr, false, [&]<typename T, int PC, class Op>(const Op& op) {
    hipLaunchKernelGGL((k_apply<T, Op>), PBCG_GRID_OP, op, x, y, S.n, S.rtiles, S.nblk);
  });
}

// y = o x for an FP64 sliced-ELL operator other than the solver's own (the
// block-Jacobi M and M^-1)
void launch_apply_op(Solver& S, const OpData& o, const double* x, double* y, hipStream_t st) {
  auto f = [&]<typename T, int PC, class Op>(const Op& op) {
    hipLaunchKernelGGL((k_apply<T, Op>), PBCG_GRID_OP, op, x, y, S.n, S.rtiles, S.nblk);
  };
  with_op_t<double>(S, o, false, f);
}

static int grid_for(int64_t count) {
  int64_t b = (count + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

void launch_grad(Solver& S, const double* lam, const double* x, double* grad, hipStream_t st) {
  switch (S.kind) {
    case OP_SELL:
      hipLaunchKernelGGL(k_grad_csr, dim3(grid_for(S.n)), dim3(kBlock), 0, st, S.d_rowptr,
                         S.d_col, lam, x, grad, S.n);
      break;
    case OP_DIA5:
      hipLaunchKernelGGL(k_grad_dia5, dim3(grid_for(S.n)), dim3(kBlock), 0, st, S.A.dims[0],
                         S.A.dims[1], lam, x, grad, S.n);
      break;
    case OP_ST2D5:
      hipLaunchKernelGGL(k_grad_st<OP_ST2D5>, PBCG_GRID_OP, S.A.dims[0], S.A.dims[1], 1, lam, x,
                         S.n, S.rtiles, S.nblk, S.partials);
      break;
    case OP_ST3D7:
      hipLaunchKernelGGL(k_grad_st<OP_ST3D7>, PBCG_GRID_OP, S.A.dims[0], S.A.dims[1], S.A.dims[2],
                         lam, x, S.n, S.rtiles, S.nblk, S.partials);
      break;
  }
}

void launch_update_sell(Solver& S, const double* val_dev, hipStream_t st) {
  int32_t* bad = &S.sc->bad_diag;
  if (S.precision == 0) {
    hipLaunchKernelGGL(k_update_sell<double>, dim3(grid_for(S.nnz)), dim3(kBlock), 0, st, val_dev,
                       S.nnz, S.d_posA, (double*)S.A.val);
    if (S.have_AT)
      hipLaunchKernelGGL(k_update_sell<double>, dim3(grid_for(S.nnz)), dim3(kBlock), 0, st,
                         val_dev, S.nnz, S.d_posAT, (double*)S.AT.val);
    if (S.precond)
      hipLaunchKernelGGL(k_update_dinv<double>, dim3(grid_for(S.n)), dim3(kBlock), 0, st, val_dev,
                         S.d_diagpos, (double*)S.dinv, S.n, bad);
  } else {
    hipLaunchKernelGGL(k_update_sell<float>, dim3(grid_for(S.nnz)), dim3(kBlock), 0, st, val_dev,
                       S.nnz, S.d_posA, (float*)S.A.val);
    if (S.have_AT)
      hipLaunchKernelGGL(k_update_sell<float>, dim3(grid_for(S.nnz)), dim3(kBlock), 0, st,
                         val_dev, S.nnz, S.d_posAT, (float*)S.AT.val);
    if (S.precond)
      hipLaunchKernelGGL(k_update_dinv<float>, dim3(grid_for(S.n)), dim3(kBlock), 0, st, val_dev,
                         S.d_diagpos, (float*)S.dinv, S.n, bad);
  }
}

void launch_kappa_assemble(Solver& S, const double* kappa, double cx, double cy, double h,
                           hipStream_t st) {
  int32_t* bad = &S.sc->bad_diag;
  const int nx = S.A.dims[0], ny = S.A.dims[1];
  if (S.precision == 0) {
    hipLaunchKernelGGL(k_kappa_assemble<double>, dim3(grid_for(S.n)), dim3(kBlock), 0, st, kappa,
                       nx, ny, cx, cy, h, (double*)S.A.dia, (double*)nullptr, S.npad,
                       (double*)S.dinv, bad);
    if (S.have_AT)
      hipLaunchKernelGGL(k_dia5_transpose<double>, dim3(grid_for(S.n)), dim3(kBlock), 0, st,
                         (const double*)S.A.dia, (double*)S.AT.dia, nx, ny, S.npad);
  } else {
    hipLaunchKernelGGL(k_kappa_assemble<float>, dim3(grid_for(S.n)), dim3(kBlock), 0, st, kappa,
                       nx, ny, cx, cy, h, (float*)S.A.dia, (float*)nullptr, S.npad,
                       (float*)S.dinv, bad);
    if (S.have_AT)
      hipLaunchKernelGGL(k_dia5_transpose<float>, dim3(grid_for(S.n)), dim3(kBlock), 0, st,
                         (const float*)S.A.dia, (float*)S.AT.dia, nx, ny, S.npad);
  }
}

void launch_kappa_grad(Solver& S, const double* lam, const double* x, double* gk,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_kappa_grad, dim3(grid_for(S.n)), dim3(kBlock), 0, st, lam, x, S.A.dims[0],
                     S.A.dims[1], gk);
}

// transpose of a DIA5 operator, used by the engine when the transpose is built
void launch_dia5_transpose(Solver& S, hipStream_t st) {
  const int nx = S.A.dims[0], ny = S.A.dims[1];
  if (S.precision == 0)
    hipLaunchKernelGGL(k_dia5_transpose<double>, dim3(grid_for(S.n)), dim3(kBlock), 0, st,
                       (const double*)S.A.dia, (double*)S.AT.dia, nx, ny, S.npad);
  else
    hipLaunchKernelGGL(k_dia5_transpose<float>, dim3(grid_for(S.n)), dim3(kBlock), 0, st,
                       (const float*)S.A.dia, (float*)S.AT.dia, nx, ny, S.npad);
}

// ----------------------------------------------------------------------------
// Algorithm 2 for small systems in one workgroup
// ----------------------------------------------------------------------------
//
// A solve of a few hundred rows is bound by kernel launches and host polls,
// not by memory.  For N <= ROWS (FP64; 1024, or 2048 with four rows per
// thread) one block of ROWS / RPT threads (RPT rows per thread) holds the
// iteration vectors (the rows of a
// thread in its registers; the inputs of the products, whose neighbours'
// entries are read, also in LDS) and runs Algorithm 2 to its end in one
// launch: phase A and phase B with the expressions of k_phaseA / k_phaseB,
// the products through the operator's own row visitor (the same terms in
// the same order), periodic residual replacement (eq:rr) in FP64 with the
// saved pre-replacement z (or with n and v refreshed, option rr_nv), and the
// termination rule: true-residual confirmation, at most three forced
// replacements, no tolerance test right after one.
//
// Two barriers per iteration.  Each global reduction stores one partial per
// wave (wave_sums_packed) before a barrier that the iteration needs anyway,
// and after it every wave adds the partials with the same moves, so every
// thread holds the same bits without a second barrier; the two products
// read M^-1 z and M^-1 w from arrays of their own, which the following
// phase does not write.  A sliced-ELL row of at most kSmallCache (with
// four rows per thread kSmallCache2k) stored
// entries is held in registers for the whole solve.

constexpr int kSmallRows = 1024;
constexpr int kSmallRowsMax = 2048;   // four rows per thread, 512 threads
constexpr int kSmallWaves = 16;       // most waves of a block (1024 threads)
static_assert(kSmallWaves == 16, "the wave partials fit one 16-lane row");
constexpr int kSmallCache = 8;
constexpr int kSmallCache2k = 5;      // with four rows per thread (2048 rows)
enum : int {
  SB_NZ = 0,  // M^-1 z_i, the input of v_i = A M^-1 z_i (also M^-1 r_0 at the start)
  SB_MW,      // M^-1 w, the input of t = A M^-1 w
  SB_PX, SB_PG, SB_PK, SB_PL,   // x, g, k, l for the products of a replacement
  SB_COUNT
};
constexpr size_t small_lds(int rows) { return (size_t)SB_COUNT * rows * sizeof(double); }
constexpr int kSmallRed = 4;          // partial buffers: GLRED 1, GLRED 2, the others, and
                                      // GLRED 1 of odd iterations (automated strategy)
constexpr int kSmallSums = 17;        // sums per buffer (automated strategy: GLRED 2 with the
                                      // norms of phase B and of a replacement)
constexpr size_t kSmallStatic = (size_t)kSmallRed * kSmallSums * kSmallWaves * sizeof(double);

struct SmallArgs {
  int n;
  const double* dinv;
  double ds;
  double* x;                 // x_0 in, the last iterate out
  const double* b;
  const double* rhat_in;     // a fixed shadow vector, or null (r_0)
  double* out[11];           // r^, r, g, s, l, z, k, w, t, v, saved z: written back at the end
  double tol, tau;
  int maxit, rr_period;
  int rr_nv;                 // a replacement also refreshes n = M^-1 z and v = A n
  double* history;
  int hist_len;
  double* bound_history;     // automated strategy: f^r per iteration, or null
  int bound_len;
  DevScalars* sc;            // the solve's scalars (the bound's constants are read from it)
};

// Workgroup sums of the single-workgroup solve: the packed wave sums of
// wave_sums_packed, one partial per wave in LDS, and after the barrier every
// wave loads the partials packed the same way, sums the rows and reads each
// total from its row (readlane), so every thread receives the same bits.
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                          __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// one partial per wave of each of NS sums
template <int NS>
__device__ __forceinline__ void small_part(const double (&v)[NS], double (*buf)[kSmallWaves]) {
  const int wv = threadIdx.x >> 6;
  wave_sums_packed<NS>(v, [&](int d, double x) { buf[d][wv] = x; });
}

// the sums of the nwaves wave partials (after a barrier): every wave loads
// them packed by row, sums the rows and reads each total from its row, so
// every thread receives the same bits
template <int NS>
__device__ __forceinline__ void small_total(double (&v)[NS], const double (*buf)[kSmallWaves],
                                            int nwaves) {
  const int lane = threadIdx.x & 63, k = lane & 15;
#pragma unroll
  for (int p = 0; p < (NS + 3) / 4; ++p) {
    const int vi = 4 * p + kRowVal[lane >> 4];
    const double t = row16_sum((vi < NS && k < nwaves) ? buf[vi < NS ? vi : 0][k] : 0.0);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (4 * p + j < NS) v[4 * p + j] = readlane_f64(t, kValLane[j]);
  }
}

// A sliced-ELL row of at most NC stored entries, in registers; the
// visit adds the entries in SellOp::row's order (ascending slot, padding
// skipped), so the sums are the same.
template <int NC>
struct SellRowRegs {
  int32_t c[NC];
  double a[NC];
  __device__ __forceinline__ void load(const SellOp<double>& op, int i) {
    const int64_t s = i >> 6;
    const int lane = i & 63;
    const int64_t off = op.sptr[s];
    const int w = (int)((op.sptr[s + 1] - off) >> 6);
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      const bool in = j < w;
      c[j] = in ? op.col[off + (int64_t)j * kSellC + lane] : -1;
      a[j] = in ? op.val[off + (int64_t)j * kSellC + lane] : 0.0;
    }
  }
  template <class Vis>
  __device__ __forceinline__ void row(Vis& vis) const {
#pragma unroll
    for (int j = 0; j < NC; ++j)
      if (c[j] >= 0) vis.add(a[j], vis.load(c[j]));
  }
};

// A sliced-ELL row of any length read from memory one entry after another,
// in SellOp::row's order; fewer registers than SellOp::row's grouped loads,
// which the register-resident vectors of k_small_solve leave no room for.
template <class Vis>
__device__ __forceinline__ void sell_row_serial(const SellOp<double>& op, int i, Vis& vis) {
  const int64_t sl = i >> 6;
  const int lane = i & 63;
  const int64_t off = op.sptr[sl];
  const int w = (int)((op.sptr[sl + 1] - off) >> 6);
  const int32_t* c = op.col + off + lane;
  const double* v = op.val + off + lane;
#pragma unroll 4
  for (int j = 0; j < w; ++j) {
    const int32_t cj = c[(int64_t)j * kSellC];
    const double aj = v[(int64_t)j * kSellC];
    if (cj >= 0) vis.add(aj, vis.load(cj));
  }
}

// RPT rows per thread: rows tid, tid + T, ... (T = ROWS / RPT threads), so
// that a wave's lanes hold consecutive rows.  AUTO: the automated strategy
// (Section 3.6, nested reading: the worst-case bound or the estimate); the
// reductions carry the norms of the bound (phase A six, phase B seven, a
// replacement five; ||y|| is GLRED 1's (y, y)); wave 0 alone advances the
// bound state (GapState) and
// passes eq:criterion's decision to the other waves through LDS.
template <int PC, class Op, bool CACHE, int RPT, bool AUTO, int ROWS>
__global__ __launch_bounds__(ROWS / RPT) void k_small_solve(Op op, SmallArgs a) {
  constexpr int T = ROWS / RPT;
  static_assert(T % 64 == 0 && T / 64 <= kSmallWaves, "waves of the block");
  constexpr int NI = AUTO ? 6 : 4;    // sums of the initialisation
  constexpr int NA = AUTO ? 8 : 2;    // GLRED 1 (+ norms), two groups of four
  constexpr int NB = AUTO ? 12 : 5;   // GLRED 2 (+ norms), three groups of four
  constexpr int NR = AUTO ? 17 : 5;   // GLRED 2 after a replacement (+ its norms)
  static_assert(NR <= kSmallSums && NA <= kSmallSums, "partial buffers");
  extern __shared__ double sm[];
  __shared__ double red[kSmallRed][kSmallSums][kSmallWaves];
  __shared__ int rr_flag;             // AUTO: eq:criterion's decision for the next iteration
  double* const nz = sm + SB_NZ * ROWS;
  double* const mw = sm + SB_MW * ROWS;
  double* const px = sm + SB_PX * ROWS;
  double* const pg = sm + SB_PG * ROWS;
  double* const pk = sm + SB_PK * ROWS;
  double* const pl = sm + SB_PL * ROWS;
  const int tid = threadIdx.x;
  const int nw = T / 64;
  int row[RPT];
  bool own[RPT];
  double di[RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    row[j] = tid + j * T;
    own[j] = row[j] < a.n;
    di[j] = (PC == PC_VECTOR && own[j]) ? a.dinv[row[j]] : 0.0;
  }
  // M^-1 u for row j of the thread (prec1's product, the diagonal in a register)
  auto prec = [&](int j, double u) {
    if (PC == PC_NONE) return u;
    if (PC == PC_SCALAR) return a.ds * u;
    return di[j] * u;
  };
  SellRowRegs<(ROWS > kSmallRows) ? kSmallCache2k : kSmallCache> rows[RPT];
  if constexpr (CACHE) {
#pragma unroll
    for (int j = 0; j < RPT; ++j)
      if (own[j]) rows[j].load(op, row[j]);
  }
  auto visit = [&](int j, auto& vis) {
    if constexpr (CACHE) rows[j].row(vis);
    else if constexpr (std::is_same_v<Op, SellOp<double>>) sell_row_serial(op, row[j], vis);
    else op.row(row[j], vis);
  };
  // sum_c a_rc in_c for row j
  auto product = [&](int j, const double* in) {
    LdsVis<double> vis{in, 0, 0.0};
    visit(j, vis);
    return vis.sum;
  };
  // the rows' entries of the iteration vectors (0 where a thread has no row);
  // m = M^-1 w and n = M^-1 z as stored for the products
  double x[RPT], bi[RPT], rh[RPT], r[RPT], g[RPT], s[RPT], l[RPT], z[RPT], k[RPT];
  double w[RPT], t[RPT], v[RPT], zs[RPT], m[RPT], n[RPT];
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    x[j] = bi[j] = rh[j] = r[j] = g[j] = s[j] = l[j] = z[j] = k[j] = 0.0;
    w[j] = t[j] = v[j] = zs[j] = m[j] = n[j] = 0.0;
  }

  // Algorithm 2 initialisation
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    if (own[j]) {
      x[j] = a.x[row[j]];
      bi[j] = a.b[row[j]];
      px[row[j]] = x[j];
    }
  }
  __syncthreads();
  double acc[NI];
#pragma unroll
  for (int e = 0; e < NI; ++e) acc[e] = 0.0;
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    if (own[j]) {
      ResVis<double> vis{px, 0.0};
      visit(j, vis);
      r[j] = bi[j] - vis.sum;
      rh[j] = a.rhat_in ? a.rhat_in[row[j]] : r[j];
      k[j] = prec(j, r[j]);
      nz[row[j]] = k[j];
      acc[0] += rh[j] * r[j];
      acc[1] += r[j] * r[j];
      acc[2] += bi[j] * bi[j];
      if constexpr (AUTO) {
        acc[4] += x[j] * x[j];
        acc[5] += k[j] * k[j];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    if (own[j]) {
      w[j] = product(j, nz);                   // w_0 = A M^-1 r_0
      m[j] = prec(j, w[j]);
      mw[row[j]] = m[j];
      acc[3] += rh[j] * w[j];
    }
  }
  small_part<NI>(acc, red[2]);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < RPT; ++j)
    if (own[j]) t[j] = product(j, mw);         // t_0 = A M^-1 w_0
  small_total<NI>(acc, red[2], nw);
  double rho = acc[0];
  const double rn0 = sqrt(acc[1]), nb = sqrt(acc[2]), rw = acc[3];
  double rn = rn0, alpha = 0.0, beta = 0.0, omega = 0.0, omega_prev = 0.0;
  int status = -1, iter = 0, rr_count = 0, forced = 0, n_saved = 0;
  if (nb == 0.0) {
    status = ST_CONVERGED;
#pragma unroll
    for (int j = 0; j < RPT; ++j) x[j] = 0.0;
  } else if (rn0 <= a.tol * nb) {
    status = ST_CONVERGED;
  } else if (!finite(rho) || !finite(rw)) {
    status = ST_NONFINITE;
  } else if (rw == 0.0) {
    status = ST_BREAKDOWN_RHO;
  } else {
    alpha = rho / rw;
  }
  // the bound of Section 3.2 at the start, and eq:criterion's previous test
  // (wave 0 holds the bound state, the other waves' gs and f_ok_prev are
  // unused; its first write of rr_flag is behind the next barrier)
  const bool bw = tid < 64;
  GapState gs;
  bool f_ok_prev = false;
  if constexpr (AUTO) {
    if (bw) {
      gs.load(a.sc);
      gs.nb = nb;
      gap_bound_start(&gs, sqrt(acc[4]), sqrt(acc[5]));
      f_ok_prev = gs.fr <= a.tau * rn0;
      if (tid == 0) rr_flag = 0;
    }
  }

  // eq:rr from x_{i+1} and g_i in FP64, and the GLRED 2 terms again (with
  // AUTO also the norms that restart the bound: x, k, l, s, z in d[12..16]).  x, g,
  // then k, l go through LDS arrays of their own (the neighbours' entries);
  // their previous readers are behind at least one barrier.
  auto replace = [&](bool save_z, double (&d)[NR]) {
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      if (own[j]) {
        px[row[j]] = x[j];
        pg[row[j]] = g[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      if (own[j]) {
        Res2Vis<double, double, double> vis{px, pg, 0.0, 0.0};
        visit(j, vis);
        r[j] = bi[j] - vis.sx;
        s[j] = vis.sy;
        k[j] = prec(j, r[j]);
        l[j] = prec(j, s[j]);
        pk[row[j]] = k[j];
        pl[row[j]] = l[j];
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 5; ++e) d[e] = 0.0;
    if constexpr (AUTO) {
#pragma unroll
      for (int e = 12; e < 17; ++e) d[e] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      if (own[j]) {
        Res2Vis<double, double, double> vis{pk, pl, 0.0, 0.0};
        visit(j, vis);
        if (save_z && !a.rr_nv) zs[j] = z[j];
        w[j] = vis.sx;
        z[j] = vis.sy;
        m[j] = prec(j, w[j]);
        mw[row[j]] = m[j];
        d[0] += rh[j] * r[j];
        d[1] += rh[j] * w[j];
        d[2] += rh[j] * s[j];
        d[3] += rh[j] * z[j];
        d[4] += r[j] * r[j];
        if constexpr (AUTO) {
          d[12] += x[j] * x[j];
          d[13] += k[j] * k[j];
          d[14] += l[j] * l[j];
          d[15] += s[j] * s[j];
          d[16] += z[j] * z[j];
        }
        if (a.rr_nv) {
          n[j] = prec(j, z[j]);
          nz[row[j]] = n[j];
        }
      }
    }
    rr_count += 1;
    n_saved = a.rr_nv ? 0 : 1;
    if (a.rr_nv) {
      // option rr_nv: v = A M^-1 z from the replaced z (the product reads the
      // rows of nz written above; the last reader of nz, the v product of this
      // iteration, is behind the barriers at the top)
      __syncthreads();
#pragma unroll
      for (int j = 0; j < RPT; ++j)
        if (own[j]) v[j] = product(j, nz);
    }
  };

  // the GLRED 2 sums (after a replacement with its norms), with `mid` and the
  // product t_{i+1} = A M^-1 w_{i+1} between the partials and the totals (the
  // norms' partials stay in red[1] for the bound)
  auto glred2_sums = [&](double (&d)[NR], bool replaced, auto&& mid) {
    constexpr int NS = AUTO ? NB : 5;
    if (replaced && AUTO) {
      small_part<NR>(d, red[1]);
    } else {
      double p[NS];
#pragma unroll
      for (int e = 0; e < NS; ++e) p[e] = d[e];
      small_part<NS>(p, red[1]);
    }
    __syncthreads();
    mid();
#pragma unroll
    for (int j = 0; j < RPT; ++j)
      if (own[j]) t[j] = product(j, mw);
    double g2[5];
    small_total<5>(g2, red[1], nw);
#pragma unroll
    for (int e = 0; e < 5; ++e) d[e] = g2[e];
  };

  // AUTO: the bound step of the iteration (eq:DDr_bound, with the norms
  // summed from the partials that phase A left in `ra` and phase B in red[1];
  // ||y||^2 is GLRED 1's (y, y), the same sum)
  // and, after a replacement, its restart from the recomputation's errors.
  // It needs alpha_i, beta_i, omega_i, omega_{i-1} and ||r_i||, not the
  // GLRED 2 totals, so it runs before the product t_{i+1} (their latencies
  // overlap); eq:criterion follows the totals.
  auto bound_update = [&](double (*rb)[kSmallWaves], double yy, bool step, bool reset) {
    if constexpr (AUTO) {
      if (!bw) return;
      double nbv[7];                           // x, u, n, v, g, s, q
      small_total<7>(nbv, red[1] + 5, nw);
      if (step) {
        double na[6];                          // k, w, t, m, l, z
        small_total<6>(na, rb + 2, nw);
        IterNorms nm;
        nm.k = sqrt(na[0]); nm.w = sqrt(na[1]); nm.t = sqrt(na[2]); nm.m = sqrt(na[3]);
        nm.l = sqrt(na[4]); nm.z = sqrt(na[5]); nm.x = sqrt(nbv[0]); nm.u = sqrt(nbv[1]);
        nm.n = sqrt(nbv[2]); nm.v = sqrt(nbv[3]); nm.g = sqrt(nbv[4]); nm.s = sqrt(nbv[5]);
        nm.q = sqrt(nbv[6]); nm.y = sqrt(yy); nm.r = rn;
        gap_bound_step(&gs, alpha, beta, omega, omega_prev, nm);
      }
      if (reset) {
        double nr[5];
        small_total<5>(nr, red[1] + 12, nw);
        gap_bound_reset(&gs, sqrt(nr[0]), sqrt(nr[1]), sqrt(nbv[4]), sqrt(nr[2]), sqrt(nr[3]),
                        sqrt(nr[4]));
      }
    }
  };

  while (status < 0) {
    // phase A: g, s, l, z, M^-1 z and the GLRED 1 terms (with AUTO the norms
    // of k, w, t, m before and of l, z after the update)
    double d2[NA];
#pragma unroll
    for (int e = 0; e < NA; ++e) d2[e] = 0.0;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      if (own[j]) {
        const double np = prec(j, n_saved ? zs[j] : z[j]);
        const double gn = k[j] + beta * (g[j] - omega_prev * l[j]);
        const double sn = w[j] + beta * (s[j] - omega_prev * z[j]);
        const double ln = m[j] + beta * (l[j] - omega_prev * np);
        const double zn = t[j] + beta * (z[j] - omega_prev * v[j]);
        const double q = r[j] - alpha * sn;
        const double y = w[j] - alpha * zn;
        d2[0] += q * y;
        d2[1] += y * y;
        if constexpr (AUTO) {
          d2[2] += k[j] * k[j];
          d2[3] += w[j] * w[j];
          d2[4] += t[j] * t[j];
          d2[5] += m[j] * m[j];
          d2[6] += ln * ln;
          d2[7] += zn * zn;
        }
        g[j] = gn; s[j] = sn; l[j] = ln; z[j] = zn;
        n[j] = prec(j, zn);
        nz[row[j]] = n[j];
      }
    }
    // With AUTO the norms' partials stay in the buffer until the bound step
    // at the end of the iteration, which no barrier separates from the next
    // phase A: consecutive iterations use two buffers.
    double (*const ra)[kSmallWaves] = (AUTO && (iter & 1)) ? red[3] : red[0];
    small_part<NA>(d2, ra);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RPT; ++j)
      if (own[j]) v[j] = product(j, nz);       // v_i = A M^-1 z_i
    double g1[2];
    small_total<2>(g1, ra, nw);                // GLRED 1
    d2[0] = g1[0];
    d2[1] = g1[1];
    n_saved = 0;
    if (!finite(d2[0]) || !finite(d2[1])) {
      status = ST_NONFINITE;
      break;
    }
    omega = d2[1] != 0.0 ? d2[0] / d2[1] : 0.0;
    // phase B: x, r, k, w, M^-1 w and the GLRED 2 terms (with AUTO the norms
    // of x before the update, u, n, v, and of phase A's g, s, q in d5[5..11];
    // q is phase A's q, the same expression of the same values)
    double d5[NR];
#pragma unroll
    for (int e = 0; e < NR; ++e) d5[e] = 0.0;
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      if (own[j]) {
        const double q = r[j] - alpha * s[j];
        const double u = k[j] - alpha * l[j];
        const double y = w[j] - alpha * z[j];
        if constexpr (AUTO) {
          d5[5] += x[j] * x[j];
          d5[6] += u * u;
          d5[7] += n[j] * n[j];
          d5[8] += v[j] * v[j];
          d5[9] += g[j] * g[j];
          d5[10] += s[j] * s[j];
          d5[11] += q * q;
        }
        x[j] = (x[j] + alpha * g[j]) + omega * u;
        const double rn_ = q - omega * y;
        const double kn = u - omega * (m[j] - alpha * n[j]);
        const double wn = y - omega * (t[j] - alpha * v[j]);
        r[j] = rn_; k[j] = kn; w[j] = wn;
        m[j] = prec(j, wn);
        mw[row[j]] = m[j];
        d5[0] += rh[j] * rn_;
        d5[1] += rh[j] * wn;
        d5[2] += rh[j] * s[j];
        d5[3] += rh[j] * z[j];
        d5[4] += rn_ * rn_;
      }
    }
    // a replacement: eq:criterion's decision of the previous iteration, or the period
    // (rr_flag was written before the last barrier, and is next written after
    // the barrier that follows this read)
    const bool due = AUTO ? rr_flag != 0
                          : (a.rr_period > 0 && (iter + 1) % a.rr_period == 0 && rn >= a.tau * rn0);
    if (due) replace(true, d5);
    glred2_sums(d5, due, [&] { bound_update(ra, d2[1], true, due); });   // GLRED 2
    const int its = ++iter;
    double* hrow = (a.history && its <= a.hist_len) ? a.history + 4 * (int64_t)(its - 1) : nullptr;
    if (hrow && tid == 0) { hrow[1] = alpha; hrow[2] = omega; hrow[3] = 0.0; }
    bool test_tol = true;
    for (;;) {
      if constexpr (AUTO)
        if (tid == 0 && a.bound_history && its <= a.bound_len) a.bound_history[its - 1] = gs.fr;
      const double g5[5] = {d5[0], d5[1], d5[2], d5[3], d5[4]};
      const G2Step st = glred2_step(g5, alpha, omega, rho, a.tol, nb, test_tol);
      if (st.outcome == G2_NONFINITE) {
        status = ST_NONFINITE;
        break;
      }
      rn = st.rn;
      if (hrow && tid == 0) hrow[0] = rn;
      if (st.outcome == G2_CONVERGED) {
        // confirm on the true residual ||b - A x|| (FP64)
#pragma unroll
        for (int j = 0; j < RPT; ++j)
          if (own[j]) px[row[j]] = x[j];
        __syncthreads();
        double tr2[1] = {0.0};
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
          if (own[j]) {
            ResVis<double> vis{px, 0.0};
            visit(j, vis);
            const double e = bi[j] - vis.sum;
            tr2[0] += e * e;
          }
        }
        small_part<1>(tr2, red[2]);
        __syncthreads();
        small_total<1>(tr2, red[2], nw);
        if (sqrt(tr2[0]) <= a.tol * nb) {
          status = ST_CONVERGED;
        } else if ((!AUTO && a.rr_period <= 0) || forced >= 3) {
          status = ST_TRUE_RES_NOT_MET;
        } else {
          // replace and go on without testing the replaced residual
          ++forced;
          replace(n_saved == 0, d5);
          glred2_sums(d5, true, [&] { bound_update(ra, d2[1], false, true); });
          test_tol = false;
          continue;
        }
      } else {
        if constexpr (AUTO) {                  // eq:criterion for the next iteration
          if (bw) {
            const bool f_ok = gs.fr <= a.tau * st.rn;
            if (tid == 0) rr_flag = (f_ok_prev && !f_ok) ? 1 : 0;
            f_ok_prev = f_ok;
          }
        }
        if (st.outcome == G2_BREAKDOWN_OMEGA) {
          status = ST_BREAKDOWN_OMEGA;
        } else if (st.outcome == G2_BREAKDOWN_RHO) {
          status = ST_BREAKDOWN_RHO;
        } else {
          beta = st.beta;
          if (hrow && tid == 0) hrow[3] = beta;
          alpha = st.alpha;
          rho = d5[0];
          omega_prev = omega;
          if (its >= a.maxit) status = ST_MAXIT;
        }
      }
      break;
    }
  }

  // write the state back: vectors, x, scalars
#pragma unroll
  for (int j = 0; j < RPT; ++j) {
    if (own[j]) {
      const int i = row[j];
      a.out[0][i] = rh[j]; a.out[1][i] = r[j]; a.out[2][i] = g[j]; a.out[3][i] = s[j];
      a.out[4][i] = l[j]; a.out[5][i] = z[j]; a.out[6][i] = k[j]; a.out[7][i] = w[j];
      a.out[8][i] = t[j]; a.out[9][i] = v[j]; a.out[10][i] = zs[j];
      a.x[i] = x[j];
    }
  }
  if (tid == 0) {
    DevScalars* sc = a.sc;
    sc->done = STOPPED;
    sc->status = status;
    sc->iter = iter;
    sc->rr_count = rr_count;
    sc->rn = rn; sc->rn0 = rn0; sc->nb = nb; sc->rho = rho;
    sc->alpha = alpha; sc->beta = beta; sc->omega = omega; sc->omega_prev = omega_prev;
    sc->n_saved = n_saved;
  }
}

template <int PC, class Op, bool CACHE, int RPT, bool AUTO, int ROWS = kSmallRows>
static hipError_t launch_small_rpt(const Op& op, const SmallArgs& a, hipStream_t st) {
  const hipError_t e =
      hipFuncSetAttribute((const void*)k_small_solve<PC, Op, CACHE, RPT, AUTO, ROWS>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)small_lds(ROWS));
  if (e == hipSuccess)
    hipLaunchKernelGGL((k_small_solve<PC, Op, CACHE, RPT, AUTO, ROWS>), dim3(1),
                       dim3(ROWS / RPT), small_lds(ROWS), st, op, a);
  return e;
}

// the automated strategy runs with two rows per thread; more than 1024 rows
// with four (512 threads, the registers of two waves per SIMD; sliced-ELL
// rows of at most kSmallCache2k entries in registers)
template <int PC, class Op, bool CACHE>
static hipError_t launch_small(const Op& op, const SmallArgs& a, int rpt, bool automated,
                               hipStream_t st) {
  if (a.n > kSmallRows) return launch_small_rpt<PC, Op, CACHE, 4, false, kSmallRowsMax>(op, a, st);
  if (automated) return launch_small_rpt<PC, Op, CACHE, 2, true>(op, a, st);
  if (rpt == 1) return launch_small_rpt<PC, Op, CACHE, 1, false>(op, a, st);
  if (rpt == 4) return launch_small_rpt<PC, Op, CACHE, 4, false>(op, a, st);
  return launch_small_rpt<PC, Op, CACHE, 2, false>(op, a, st);
}

bool launch_small_solve(Solver& S, const pbcg_opts& o, hipStream_t st, hipError_t* err) {
  // the products reading of the automated strategy (rr_auto 3, 4) keeps a
  // state per error source in a caller's buffer: not here; nor the automated
  // strategy above 1024 rows (its registers with four rows per thread)
  const int rows = S.n > kSmallRows ? kSmallRowsMax : kSmallRows;
  if (S.n > kSmallRowsMax || (S.n > kSmallRows && o.rr_auto) || S.precision != 0 ||
      o.transpose || o.rr_auto > 2 || o.gap_every > 0 || o.restarts > 0 || S.block ||
      (size_t)S.lds_cap < small_lds(rows) + kSmallStatic)
    return false;
  SmallArgs a{};
  a.n = (int)S.n;
  a.dinv = (const double*)S.dinv;
  a.ds = S.dinv_s;
  a.x = S.x;
  a.b = S.b;
  a.rhat_in = o.rhat;
  const int ids[11] = {V_RHAT, V_R, V_G, V_S, V_L, V_Z, V_K, V_W, V_T, V_V, V_TMP};
  for (int c = 0; c < 11; ++c) a.out[c] = (double*)S.vec[ids[c]];
  a.tol = o.tol;
  a.tau = S.h_sc[2].tau;      // the scalars begin_solve uploaded (automated: sqrt(eps))
  a.maxit = o.maxit;
  a.rr_period = o.rr_period;
  a.rr_nv = o.rr_nv ? 1 : 0;
  a.history = o.history;
  a.hist_len = o.history ? o.history_len : 0;
  a.bound_history = o.rr_auto ? o.bound_history : nullptr;
  a.bound_len = a.bound_history ? o.bound_len : 0;
  a.sc = S.sc;
  // rows of the sliced-ELL operator short enough to stay in registers
  const bool cache = S.mu_row <= (S.n > kSmallRows ? kSmallCache2k : kSmallCache);
  const int rpt = S.small_rpt;
  with_op(S, false, true, [&]<typename T, int PC, class Op>(const Op& op) {
    if constexpr (std::is_same_v<T, double>) {
      if constexpr (std::is_same_v<Op, SellOp<double>>) {
        *err = cache ? launch_small<PC, Op, true>(op, a, rpt, o.rr_auto != 0, st)
                     : launch_small<PC, Op, false>(op, a, rpt, o.rr_auto != 0, st);
      } else {
        *err = launch_small<PC, Op, false>(op, a, rpt, o.rr_auto != 0, st);
      }
    }
  });
  return true;
}

}  // namespace pbcg
