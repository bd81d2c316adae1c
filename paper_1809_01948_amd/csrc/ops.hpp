// Sparse operators of the library, as row visitors.
//
// Each operator exposes `row(i, vis)`.  A visitor provides
//   V load(j)        the input value(s) needed from column j, and
//   add(a_ij, v)     accumulation of one stored entry,
// and the operator calls add() for the stored entries of row i in ascending
// column order.  Every load of a row is issued before the first add (loads of
// entries that do not exist are redirected to the row itself and their adds
// skipped), so a row costs one memory round trip instead of one per entry.
// Summing in ascending column order, one rounding per multiply and per add
// (the library is compiled without FMA contraction), reproduces a sequential
// CSR product exactly.
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
  // entries whose loads are issued together: nine (the 2e6 x 27 random
  // matrix's product 231 -> 212 us against eight; sixteen, or eight waves per
  // SIMD, were slower: the gathers' L1 hit rate falls)
  static constexpr int kGroup = 9;
  template <class Vis>
  __device__ __forceinline__ void row(int64_t i, Vis& vis) const {
    const int64_t s = i >> 6;
    const int lane = (int)(i & 63);
    const int64_t off = sptr[s];
    const int w = (int)((sptr[s + 1] - off) >> 6);
    const int32_t* c = col + off + lane;
    const T* a = val + off + lane;
    for (int j0 = 0; j0 < w; j0 += kGroup) {
      int32_t cj[kGroup];
      T aj[kGroup];
#pragma unroll
      for (int u = 0; u < kGroup; ++u) {
        const int jj = min(j0 + u, w - 1);
        // the matrix streams through once: non-temporal, so that the L2 keeps
        // the gathered x (2e6 x 27 random matrix: 212 -> 204 us FP64, 146 ->
        // 141 us FP32 storage)
        cj[u] = __builtin_nontemporal_load(c + (int64_t)jj * kSellC);
        aj[u] = __builtin_nontemporal_load(a + (int64_t)jj * kSellC);
      }
      typename Vis::V xv[kGroup];
#pragma unroll
      for (int u = 0; u < kGroup; ++u) xv[u] = vis.load(cj[u] >= 0 ? (int64_t)cj[u] : i);
#pragma unroll
      for (int u = 0; u < kGroup; ++u)
        if (j0 + u < w && cj[u] >= 0) vis.add(aj[u], xv[u]);
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
    const bool hS = iy > 0, hW = ix > 0, hE = ix < nx - 1, hN = iy < ny - 1;
    const auto xS = vis.load((int64_t)(hS ? p - nx : p));
    const auto xW = vis.load((int64_t)(hW ? p - 1 : p));
    const auto xC = vis.load((int64_t)p);
    const auto xE = vis.load((int64_t)(hE ? p + 1 : p));
    const auto xN = vis.load((int64_t)(hN ? p + nx : p));
    if (hS) vis.add(c[0], xS);
    if (hW) vis.add(c[1], xW);
    vis.add(c[2], xC);
    if (hE) vis.add(c[3], xE);
    if (hN) vis.add(c[4], xN);
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
    const bool hD = iz > 0, hS = iy > 0, hW = ix > 0, hE = ix < nx - 1, hN = iy < ny - 1,
               hU = iz < nz - 1;
    const auto xD = vis.load((int64_t)(hD ? p - nxy : p));
    const auto xS = vis.load((int64_t)(hS ? p - nx : p));
    const auto xW = vis.load((int64_t)(hW ? p - 1 : p));
    const auto xC = vis.load((int64_t)p);
    const auto xE = vis.load((int64_t)(hE ? p + 1 : p));
    const auto xN = vis.load((int64_t)(hN ? p + nx : p));
    const auto xU = vis.load((int64_t)(hU ? p + nxy : p));
    if (hD) vis.add(c[0], xD);
    if (hS) vis.add(c[1], xS);
    if (hW) vis.add(c[2], xW);
    vis.add(c[3], xC);
    if (hE) vis.add(c[4], xE);
    if (hN) vis.add(c[5], xN);
    if (hU) vis.add(c[6], xU);
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
    const bool hS = iy > 0, hW = ix > 0, hE = ix < nx - 1, hN = iy < ny - 1;
    const T cS = dia[i], cW = dia[ld + i], cC = dia[2 * ld + i], cE = dia[3 * ld + i],
            cN = dia[4 * ld + i];
    const auto xS = vis.load((int64_t)(hS ? p - nx : p));
    const auto xW = vis.load((int64_t)(hW ? p - 1 : p));
    const auto xC = vis.load((int64_t)p);
    const auto xE = vis.load((int64_t)(hE ? p + 1 : p));
    const auto xN = vis.load((int64_t)(hN ? p + nx : p));
    if (hS) vis.add(cS, xS);
    if (hW) vis.add(cW, xW);
    vis.add(cC, xC);
    if (hE) vis.add(cE, xE);
    if (hN) vis.add(cN, xN);
  }
};

// ----------------------------------------------------------------------------
// structured operators, several consecutive rows per thread
// ----------------------------------------------------------------------------

// (M^-1 z)_j for the compile-time preconditioner kind
template <typename T, int PC>
__device__ __forceinline__ T prec1(T zj, const T* __restrict__ dinv, T ds, int64_t j) {
  if (PC == PC_NONE) return zj;
  if (PC == PC_SCALAR) return ds * zj;
  return dinv[j] * zj;
}

// one 16-byte chunk of M^-1 z starting at element j
template <typename T, int PC>
__device__ __forceinline__ void load_chunk(const T* __restrict__ z, const T* __restrict__ dinv, T ds,
                                           int64_t j, T (&v)[V16<T>::n]) {
  ld16(z + j, v);
  if (PC == PC_SCALAR) {
#pragma unroll
    for (int e = 0; e < V16<T>::n; ++e) v[e] = ds * v[e];
  } else if (PC == PC_VECTOR) {
    T d[V16<T>::n];
    ld16(dinv + j, d);
#pragma unroll
    for (int e = 0; e < V16<T>::n; ++e) v[e] = d[e] * v[e];
  }
}

template <typename T>
struct StParams {
  int kind;          // OP_ST2D5, OP_ST3D7 or OP_DIA5
  int nx, ny, nz;
  T c[7];            // constant coefficients (ascending column order)
  const T* __restrict__ dia;
  int64_t ld;
  int mz;            // phase kernels: planes per work item of the plane march (0: row order)
};

// The order in which a phase kernel's block visits its tiles.  Row order
// (mz == 0): tiles of kBlock * C consecutive rows, XCD-aware (XcdWalk).
// Plane march (3D grids): work items (z-chunk of mz planes, segment of
// kBlock * C rows of one plane), XCD-aware over the items, an item's planes
// in ascending order, so that a tile's neighbours a plane away are the
// previous and next tiles of the same item; in the last segment of a plane
// the threads past the plane's end have no row (`has`).
struct TileSeq {
  int64_t t, end, step;    // tiles (row order) or items (march) of this block
  int64_t r;               // this thread's first row of the current tile
  int mz, nz, nxy, ncol, seg, k, z1;
  bool has;
  bool cont;               // march: this tile is the next plane of the previous tile's item
  __device__ TileSeq(int64_t ntiles, int C, int nx, int ny, int nz_, int mz_) {
    mz = mz_;
    nz = nz_;
    seg = kBlock * C;
    if (mz > 0) {
      nxy = nx * ny;
      ncol = (nxy + seg - 1) / seg;
      const int64_t items = (int64_t)ncol * ((nz + mz - 1) / mz);
      const XcdWalk w(items, blockIdx.x, gridDim.x);
      t = w.t; end = w.end; step = w.step;
      if (t < end) start_item();
    } else {
      const XcdWalk w(ntiles, blockIdx.x, gridDim.x);
      t = w.t; end = w.end; step = w.step;
      r = (t * kBlock + threadIdx.x) * C;
      has = true;
    }
    cont = false;
  }
  __device__ void start_item() {
    const int zc = (int)(t / ncol);
    const int c = (int)(t - (int64_t)zc * ncol);
    const int off = c * seg + (int)threadIdx.x * (seg / kBlock);
    k = zc * mz;
    z1 = k + mz < nz ? k + mz : nz;
    has = off < nxy;
    r = (int64_t)k * nxy + off;
    cont = false;
  }
  __device__ int64_t row() const { return r; }
  __device__ bool valid() const { return t < end; }
  __device__ void next() {
    if (mz > 0) {
      if (++k < z1) {
        r += nxy;
        cont = true;
        return;
      }
      t += step;
      if (t < end) start_item();
    } else {
      t += step;
      r += (int64_t)step * seg;
    }
  }
};

// Row order alone (the kernels that never march: 2D and DIA5 products), the
// interface of TileSeq with the row computed from the tile index
struct RowSeq {
  int64_t t, end, step;
  int C;
  static constexpr bool has = true;
  static constexpr bool cont = false;
  __device__ RowSeq(int64_t ntiles, int C_) : C(C_) {
    const XcdWalk w(ntiles, blockIdx.x, gridDim.x);
    t = w.t; end = w.end; step = w.step;
  }
  __device__ int64_t row() const { return (t * kBlock + threadIdx.x) * C; }
  __device__ bool valid() const { return t < end; }
  __device__ void next() { t += step; }
};

// One row of a structured operator applied to preconditioned values: the
// stored entries in ascending column order (D, S, W, C, E, N, U in 3D; S, W,
// C, E, N in 2D), one rounding per operation; entries outside the grid are
// skipped.  Every structured product (st_apply, the plane-marching 3D
// SpMV) sums through this function, so they agree bit for bit.
template <typename T, int KIND>
__device__ __forceinline__ T st_row_sum(const StParams<T>& P, bool hD, bool hS, bool vw, bool ve,
                                        bool hN, bool hU, T xd, T xs, T xw, T xc, T xe, T xn,
                                        T xu, T cS, T cW, T cC, T cE, T cN) {
  T sum = T(0);
  if (KIND == OP_DIA5) {
    if (hS) sum += cS * xs;
    if (vw) sum += cW * xw;
    sum += cC * xc;
    if (ve) sum += cE * xe;
    if (hN) sum += cN * xn;
  } else if (KIND == OP_ST3D7) {
    if (hD) sum += P.c[0] * xd;
    if (hS) sum += P.c[1] * xs;
    if (vw) sum += P.c[2] * xw;
    sum += P.c[3] * xc;
    if (ve) sum += P.c[4] * xe;
    if (hN) sum += P.c[5] * xn;
    if (hU) sum += P.c[6] * xu;
  } else {
    if (hS) sum += P.c[0] * xs;
    if (vw) sum += P.c[1] * xw;
    sum += P.c[2] * xc;
    if (ve) sum += P.c[3] * xe;
    if (hN) sum += P.c[4] * xn;
  }
  return sum;
}

// Rows p .. p + R*CH - 1 of A M^-1 z for a structured operator (constant 2D
// 5-point or 3D 7-point stencil, or DIA5), R = elements per 16-byte chunk.
// The caller passes the centre values xc = (M^-1 z)[p ..] it already holds;
// the neighbours are loaded here.  Requires p < n and nx a multiple of R, so
// that a chunk never crosses a grid line.  Each row is summed in ascending
// column order with one rounding per operation, which is the CSR product of
// the same matrix bit for bit; the result does not depend on CH or on which
// kernel calls this.
// NTC: the DIA5 coefficient rows are loaded non-temporally (FP64 kernels
// whose vector streams are: 2048^2 DIA5 phase kernels 120 -> 100 us and
// 132 -> 111 us; with FP32 storage cached loads were faster, 47 -> 51 us).
template <typename T, int PC, int KIND, int CH, bool NTC = false>
__device__ __forceinline__ void st_apply(const StParams<T>& P, const T* __restrict__ z,
                                         const T* __restrict__ dinv, T ds, int p,
                                         const T (&xc)[V16<T>::n * CH],
                                         T (&res)[V16<T>::n * CH]) {
  constexpr int R = V16<T>::n;
  constexpr int RR = R * CH;
  constexpr bool THREE = KIND == OP_ST3D7;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int nxy = nx * ny;
  int ix, iy, iz = 0;
  if (THREE) {
    iz = p / nxy;
    const int rem = p - iz * nxy;
    iy = rem / nx;
    ix = rem - iy * nx;
  } else {
    iy = p / nx;
    ix = p - iy * nx;
  }
  // neighbours outside the grid are redirected to row p itself (in bounds)
  // and their terms skipped
  const bool hS = iy > 0, hN = iy < ny - 1;
  const bool hD = THREE && iz > 0, hU = THREE && iz < nz - 1;
  const bool hW0 = ix > 0, hEl = ix + RR < nx;
  T xs[RR], xn[RR], xd[RR], xu[RR];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    T t[R];
    load_chunk<T, PC>(z, dinv, ds, (hS ? p - nx : p) + c * R, t);
#pragma unroll
    for (int e = 0; e < R; ++e) xs[c * R + e] = t[e];
    load_chunk<T, PC>(z, dinv, ds, (hN ? p + nx : p) + c * R, t);
#pragma unroll
    for (int e = 0; e < R; ++e) xn[c * R + e] = t[e];
    if (THREE) {
      load_chunk<T, PC>(z, dinv, ds, (hD ? p - nxy : p) + c * R, t);
#pragma unroll
      for (int e = 0; e < R; ++e) xd[c * R + e] = t[e];
      load_chunk<T, PC>(z, dinv, ds, (hU ? p + nxy : p) + c * R, t);
#pragma unroll
      for (int e = 0; e < R; ++e) xu[c * R + e] = t[e];
    }
  }
  const int jw = hW0 ? p - 1 : p, je = hEl ? p + RR : p;
  const T xw0 = prec1<T, PC>(z[jw], dinv, ds, jw);
  const T xeR = prec1<T, PC>(z[je], dinv, ds, je);
  T cS[RR], cW[RR], cC[RR], cE[RR], cN[RR];
  if (KIND == OP_DIA5) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      T t[R];
      const int64_t q = p + c * R;
      ldc<T, R, NTC>(P.dia + q, t);
#pragma unroll
      for (int e = 0; e < R; ++e) cS[c * R + e] = t[e];
      ldc<T, R, NTC>(P.dia + P.ld + q, t);
#pragma unroll
      for (int e = 0; e < R; ++e) cW[c * R + e] = t[e];
      ldc<T, R, NTC>(P.dia + 2 * P.ld + q, t);
#pragma unroll
      for (int e = 0; e < R; ++e) cC[c * R + e] = t[e];
      ldc<T, R, NTC>(P.dia + 3 * P.ld + q, t);
#pragma unroll
      for (int e = 0; e < R; ++e) cE[c * R + e] = t[e];
      ldc<T, R, NTC>(P.dia + 4 * P.ld + q, t);
#pragma unroll
      for (int e = 0; e < R; ++e) cN[c * R + e] = t[e];
    }
  }
#pragma unroll
  for (int e = 0; e < RR; ++e) {
    const T xw = e == 0 ? xw0 : xc[e - 1];
    const T xe = e == RR - 1 ? xeR : xc[e + 1];
    const bool vw = e == 0 ? hW0 : true;
    const bool ve = e == RR - 1 ? hEl : true;
    res[e] = st_row_sum<T, KIND>(P, hD, hS, vw, ve, hN, hU, THREE ? xd[e] : T(0), xs[e], xw,
                                 xc[e], xe, xn[e], THREE ? xu[e] : T(0),
                                 KIND == OP_DIA5 ? cS[e] : T(0), KIND == OP_DIA5 ? cW[e] : T(0),
                                 KIND == OP_DIA5 ? cC[e] : T(0), KIND == OP_DIA5 ? cE[e] : T(0),
                                 KIND == OP_DIA5 ? cN[e] : T(0));
  }
}

// The 3D 7-point product of one chunk whose neighbours a plane below and
// above are given (preconditioned, xd and xu: the plane march carries them in
// registers); the grid-line and row neighbours are loaded as in st_apply.
// Sums through st_row_sum, so the result equals st_apply's bit for bit.
template <typename T, int PC>
__device__ __forceinline__ void st_apply3_planes(const StParams<T>& P, const T* __restrict__ z,
                                                 const T* __restrict__ dinv, T ds, int p,
                                                 const T (&xd)[V16<T>::n],
                                                 const T (&xc)[V16<T>::n],
                                                 const T (&xu)[V16<T>::n],
                                                 T (&res)[V16<T>::n]) {
  constexpr int R = V16<T>::n;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  const int nxy = nx * ny;
  const int iz = p / nxy;
  const int rem = p - iz * nxy;
  const int iy = rem / nx;
  const int ix = rem - iy * nx;
  const bool hS = iy > 0, hN = iy < ny - 1;
  const bool hD = iz > 0, hU = iz < nz - 1;
  const bool hW0 = ix > 0, hEl = ix + R < nx;
  T xs[R], xn[R];
  load_chunk<T, PC>(z, dinv, ds, hS ? p - nx : p, xs);
  load_chunk<T, PC>(z, dinv, ds, hN ? p + nx : p, xn);
  const int jw = hW0 ? p - 1 : p, je = hEl ? p + R : p;
  const T xw0 = prec1<T, PC>(z[jw], dinv, ds, jw);
  const T xeR = prec1<T, PC>(z[je], dinv, ds, je);
#pragma unroll
  for (int e = 0; e < R; ++e) {
    const T xw = e == 0 ? xw0 : xc[e - 1];
    const T xe = e == R - 1 ? xeR : xc[e + 1];
    const bool vw = e == 0 ? hW0 : true;
    const bool ve = e == R - 1 ? hEl : true;
    res[e] = st_row_sum<T, OP_ST3D7>(P, hD, hS, vw, ve, hN, hU, xd[e], xs[e], xw, xc[e], xe,
                                     xn[e], xu[e], T(0), T(0), T(0), T(0), T(0));
  }
}

// ----------------------------------------------------------------------------
// final reductions (one block)
// ----------------------------------------------------------------------------

__device__ __forceinline__ void stop(DevScalars* sc, int status) {
  sc->done = STOPPED;
  sc->status = status;
}

// ----------------------------------------------------------------------------
// automated residual replacement: the running bound f^r (Section 3.6)
// ----------------------------------------------------------------------------
//
// Local errors of iteration i bounded as in eq:errbounds1-4 (epsilon eps_b,
// mu = max nonzeros per row, mu~ = 1 for a diagonal M^-1, ||A||, ||M^-1||
// upper bounds), gap norms by the triangle inequality on eq:Ds, eq:Dw, eq:Dz,
// accumulated into f^r as in eq:DDr_bound.  All evaluated left to right in
// FP64 by one thread.

struct IterNorms {
  double x, g, u, q, y, r, s, k, l, w, z, m, t, n, v;
};

// Bounds of the local rounding errors of iteration i (eq:errbounds1-4).
// a, b, w, wp are |alpha_i|, |beta_i|, |omega_i|, |omega_{i-1}|.
struct LocalBounds {
  double x, r, q, u, y, g, s, l, z, k, w;
};
// The bound functions take the scalar struct or any state with the same
// fields (the single-workgroup solve keeps one in registers; St::kProducts
// false: the nested reading only).  The factors of the products' rounding
// errors, mu sqrt(N) (worst case) or sqrt(mu) (estimate) and 1 or sqrt(N):
// a state that holds them (cmu, cnu) gives them, else they are computed.
template <class St>
__device__ inline double gap_cmu(const St* sc) {
  if constexpr (requires { sc->cmu; }) return sc->cmu;
  else return sc->rr_est ? sqrt(sc->mu) : sc->mu * sqrt(sc->nN);
}
template <class St>
__device__ inline double gap_cnu(const St* sc) {
  if constexpr (requires { sc->cnu; }) return sc->cnu;
  else return sc->rr_est ? 1.0 : sqrt(sc->nN);
}

template <class St>
__device__ inline LocalBounds gap_local_bounds(const St* sc, double a, double b, double w,
                                               double wp, const IterNorms& nm) {
  const double e = sc->eps_b, nA = sc->nA;
  const double smu = gap_cmu(sc) * nA;
  const double smut = gap_cnu(sc) * sc->nM;
  LocalBounds d;
  d.x = (2 * nm.x + 3 * a * nm.g + 2 * w * nm.u) * e;
  d.r = (nm.q + 2 * w * nm.y) * e;
  d.q = (nm.r + 2 * a * nm.s) * e;
  d.u = (nm.k + 2 * a * nm.l) * e;
  d.y = (nm.w + 2 * a * nm.z) * e;
  d.g = (nm.k + 3 * b * sc->pg + 4 * b * wp * sc->pl) * e;
  d.s = (nm.w + 3 * b * sc->ps + 4 * b * wp * sc->pz) * e;
  d.l = (nm.m + smut * nm.w + 3 * b * sc->pl + 4 * b * wp * sc->pn + smut * b * wp * sc->pz) * e;
  d.z = (nm.t + smu * nm.m + smut * nA * nm.w + 3 * b * sc->pz + 4 * b * wp * sc->pv +
         smu * b * wp * sc->pn + smut * nA * b * wp * sc->pz) * e;
  d.k = (nm.u + 3 * w * nm.m + smut * w * nm.w + 4 * w * a * nm.n + smut * w * a * nm.z) * e;
  d.w = (nm.y + 3 * w * nm.t + smu * w * nm.m + smut * nA * w * nm.w + 4 * w * a * nm.v +
         smu * w * a * nm.n + smut * nA * w * a * nm.z) * e;
  return d;
}

// One iteration of the bound.  Nested reading: f^r_{i+1} from the running
// gap-norm bounds (eq:DDr_bound as printed).  Products reading: the bounds of
// the local error groups entering the r, w, s and z gaps (eq:Dr, eq:Dw,
// eq:Ds, eq:Dz) and the signed scalars are handed to k_bound_products.
template <class St>
__device__ inline void gap_bound_step(St* sc, double as, double bs, double ws,
                                      double wps, const IterNorms& nm) {
  const double a = fabs(as), b = fabs(bs), w = fabs(ws), wp = fabs(wps);
  const LocalBounds d = gap_local_bounds(sc, a, b, w, wp, nm);
  const double e = sc->eps_b, nA = sc->nA;
  const double smu = gap_cmu(sc) * nA;
  bool prod = false;
  if constexpr (St::kProducts) prod = sc->gb_prod;
  if (prod) {
    if constexpr (St::kProducts) {
      sc->pr_a = as; sc->pr_b = bs; sc->pr_w = ws; sc->pr_wp = wps;
      sc->pr_R = nA * d.x + d.r + w * nA * d.u + d.q + w * d.y;
      sc->pr_W = nA * d.k + d.w + nA * d.u + d.y;
      sc->pr_S = nA * d.g + d.s;
      sc->pr_Z = nA * d.l + d.z;
      sc->pr_S0 = smu * nm.g * e;
      sc->pr_Z0 = smu * nm.l * e;
      sc->pr_op |= PR_STEP;
    }
  } else {
    double dz, ds;
    if (sc->gb_first) {   // Delta^s_0, Delta^z_0: the initial gaps of Section 3.2 (g_0 = k_0, l_0 = m_0)
      ds = smu * nm.g * e;
      dz = smu * nm.l * e;
      sc->gb_first = 0;
    } else {
      dz = b * sc->dz_prev + nA * d.l + d.z;                                    // eq:Dz
      ds = sc->dw + b * sc->ds_prev + b * wp * sc->dz_prev + nA * d.g + d.s;    // eq:Ds
    }
    const double f = sc->fr + a * ds + w * sc->dw + w * a * dz + nA * d.x + d.r +   // eq:Dr
                     w * nA * d.u + d.q + w * d.y;
    const double dw = sc->dw + a * dz + nA * d.k + d.w + nA * d.u + d.y;             // eq:Dw
    sc->fr = f; sc->dw = dw; sc->ds_prev = ds; sc->dz_prev = dz;
  }
  sc->pg = nm.g; sc->ps = nm.s; sc->pl = nm.l; sc->pz = nm.z; sc->pn = nm.n; sc->pv = nm.v;
}

// Bounds at the start of Algorithm 2 (Section 3.2): ||Delta^r_0|| <=
// ((mu sqrt(N) + 1) ||A|| ||x_0|| + ||b||) eps, ||Delta^w_0|| <= mu sqrt(N)
// ||A|| ||k_0|| eps; the s and z gaps of iteration 0 are set by its step.
template <class St>
__device__ inline void gap_bound_start(St* sc, double nx, double nk) {
  const double e = sc->eps_b;
  const double cmu = gap_cmu(sc);
  sc->fr = ((cmu + 1.0) * sc->nA * nx + sc->nb) * e;
  sc->dw = cmu * sc->nA * nk * e;
  sc->ds_prev = sc->dz_prev = 0.0;
  sc->gb_first = 1;
  sc->pg = sc->ps = sc->pl = sc->pz = sc->pn = sc->pv = 0.0;
  if constexpr (St::kProducts)
    if (sc->gb_prod) sc->pr_op = PR_START;  // column 0: the initial r and w gaps (fr, dw)
}

// bounds right after an explicit recomputation of r, k, w from x and s, l, z
// from g, in the arithmetic of the recomputation (FP64: eps_r); the next
// step's local bounds use the replaced s, l, z
template <class St>
__device__ inline void gap_bound_reset(St* sc, double nx, double nk, double ng, double nl,
                                       double ns, double nz) {
  const double e = sc->eps_r;
  const double cmu = gap_cmu(sc);
  const double smu = cmu * sc->nA;
  sc->fr = ((cmu + 1.0) * sc->nA * nx + sc->nb) * e;
  sc->dw = smu * nk * e;
  sc->ds_prev = smu * ng * e;
  sc->dz_prev = smu * nl * e;
  sc->gb_first = 0;
  sc->pl = nl;
  sc->ps = ns;
  sc->pz = nz;
  if constexpr (St::kProducts) {
    if (sc->gb_prod) {    // a new system: these gaps in columns 1 (r, w) and 0 (s, z)
      sc->pr_rR = sc->fr; sc->pr_rW = sc->dw; sc->pr_rS = sc->ds_prev; sc->pr_rZ = sc->dz_prev;
      sc->pr_op |= PR_RESET;
    }
  }
}

// The nested reading's state and constants, for a solve that keeps them in
// registers (every thread the same values).
struct GapState {
  static constexpr bool kProducts = false;
  int rr_est, gb_first;
  double eps_b, eps_r, nA, nM, mu, nN, nb;
  double cmu, cnu;                 // gap_cmu, gap_cnu of the constants above
  double fr, dw, ds_prev, dz_prev;
  double pg, ps, pl, pz, pn, pv;
  __device__ void load(const DevScalars* s) {
    rr_est = s->rr_est;
    gb_first = 1;
    eps_b = s->eps_b; eps_r = s->eps_r;
    nA = s->nA; nM = s->nM; mu = s->mu; nN = s->nN;
    cmu = rr_est ? sqrt(mu) : mu * sqrt(nN);
    cnu = rr_est ? 1.0 : sqrt(nN);
    nb = 0.0;
    fr = dw = ds_prev = dz_prev = 0.0;
    pg = ps = pl = pz = pn = pv = 0.0;
  }
};

// Slots each final mode reduces.  GLRED 2 in automated mode adds the norms
// of the gap bound; FIN_SUM reduces slots 0 .. aux-1.
constexpr int kMaxFinSlots = 24;

struct FinSlots {
  int n;
  int s[kMaxFinSlots];
};

__host__ __device__ inline FinSlots fin_slots(int mode, int rr_auto, int aux) {
  FinSlots f{};
  auto put = [&f](int slot) { f.s[f.n++] = slot; };
  switch (mode) {
    case FIN_INIT:
      put(SL_RR0); put(SL_RW0); put(SL_RR); put(SL_BB); put(SL_X2); put(SL_K2);
      break;
    case FIN_OMEGA:
    case FIN_C_OMEGA:
      put(SL_QY); put(SL_YY);
      break;
    case FIN_BETA:
    case FIN_REDO:
    case FIN_PROBE:
      put(SL_RR0); put(SL_RW0); put(SL_RS0); put(SL_RZ0); put(SL_RR);
      if (rr_auto && mode != FIN_PROBE) {
        put(SL_K2); put(SL_W2); put(SL_T2); put(SL_M2); put(SL_G2); put(SL_S2); put(SL_L2);
        put(SL_Z2); put(SL_Q2); put(SL_Y2); put(SL_X2); put(SL_U2); put(SL_N2); put(SL_V2);
        put(SL_RX2); put(SL_RK2); put(SL_RL2); put(SL_RS2); put(SL_RZ2);
      }
      break;
    case FIN_TRUE:
    case FIN_GAP:
      put(SL_RR);
      break;
    case FIN_C_INIT:
      put(SL_RR0); put(SL_RR); put(SL_BB);
      break;
    case FIN_C_ALPHA:
      put(SL_RS0);
      break;
    case FIN_C_BETA:
      put(SL_RR0); put(SL_RR);
      break;
    case FIN_SUM:
      for (int j = 0; j < aux && j < 8; ++j) put(j);
      break;
    default:
      break;
  }
  return f;
}

// number of slots a final mode reduces
__host__ __device__ inline int fin_slot_count(int mode, int rr_auto) {
  return fin_slots(mode, rr_auto, 8).n;
}

// The scalar step of GLRED 2 without side effects: from the reduced sums
// v = {(r0, r_{i+1}), (r0, w_{i+1}), (r0, s_i), (r0, z_i), (r_{i+1}, r_{i+1})}
// and the current alpha_i, omega_i, rho_i, the stopping test and
// beta_{i+1} = ((alpha_i / omega_i) rho_{i+1}) / rho_i,
// alpha_{i+1} = rho_{i+1} / ((r0,w_{i+1}) + beta (r0,s_i) - (beta omega_i) (r0,z_i)).
// run_final(FIN_BETA) applies it to the scalar struct; the phase A prologue
// evaluates it in every thread.
enum G2Outcome : int { G2_CONTINUE = 0, G2_NONFINITE, G2_CONVERGED, G2_BREAKDOWN_OMEGA,
                       G2_BREAKDOWN_RHO };
struct G2Step {
  int outcome;
  double rn, beta, alpha;
};
__device__ __forceinline__ G2Step glred2_step(const double (&v)[5], double alpha, double omega,
                                              double rho, double tol, double nb,
                                              bool test_tol = true) {
  G2Step r{G2_CONTINUE, 0.0, 0.0, 0.0};
  const double rho1 = v[0], rw = v[1], rs = v[2], rz = v[3], rr = v[4];
  if (!finite(rho1) || !finite(rw) || !finite(rs) || !finite(rz) || !finite(rr)) {
    r.outcome = G2_NONFINITE;
    return r;
  }
  r.rn = sqrt(rr);
  if (test_tol && r.rn <= tol * nb) {
    r.outcome = G2_CONVERGED;
  } else if (omega == 0.0) {
    r.outcome = G2_BREAKDOWN_OMEGA;
  } else if (rho1 == 0.0 || rho == 0.0) {
    r.outcome = G2_BREAKDOWN_RHO;
  } else {
    r.beta = ((alpha / omega) * rho1) / rho;
    const double den = (rw + r.beta * rs) - (r.beta * omega) * rz;
    if (den == 0.0) r.outcome = G2_BREAKDOWN_RHO;
    else r.alpha = rho1 / den;
  }
  return r;
}

// NS sums of a final, already reduced and stored in pre[] by slot
template <int NS>
__device__ __forceinline__ void take_sums(const double* pre, const int (&sl)[NS], double (&v)[NS]) {
#pragma unroll
  for (int d = 0; d < NS; ++d) v[d] = pre[sl[d]];
}

// Runs the scalar logic of one final mode on the sums in pre[] (indexed by
// slot).  Executed by one thread.
__device__ inline void run_final(int mode, DevScalars* __restrict__ sc, const double* pre, int aux) {
  switch (mode) {
    case FIN_INIT: {
      // Algorithm 2 initialisation: rho_0 = (r0, r0), alpha_0 = rho_0 / (r0, w0)
      const int sl[6] = {SL_RR0, SL_RW0, SL_RR, SL_BB, SL_X2, SL_K2};
      double v[6];
      take_sums<6>(pre, sl, v);
      const double rho = v[0], rw = v[1], rr = v[2], bb = v[3];
      {
        sc->sig[SL_RR0] = rho; sc->sig[SL_RW0] = rw; sc->sig[SL_RR] = rr; sc->sig[SL_BB] = bb;
        sc->rho = rho;
        sc->rn0 = sqrt(rr);
        sc->rn = sc->rn0;
        sc->nb = sqrt(bb);
        sc->beta = 0.0;
        sc->omega = 0.0;
        sc->omega_prev = 0.0;
        sc->n_saved = 0;                       // the iteration count is set by the host
        if (sc->rr_auto) {
          gap_bound_start(sc, sqrt(v[4]), sqrt(v[5]));
          sc->f_ok_prev = sc->fr <= sc->tau * sc->rn0;
          sc->rr_next = 0;
          sc->rr_hit = 0;
        }
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
      const int sl[2] = {SL_QY, SL_YY};
      double v[2];
      take_sums<2>(pre, sl, v);
      const double s1 = v[0], s2 = v[1];
      {
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
      // In automated mode the norms of the bound are reduced in the same pass.
      constexpr int NS = 24;
      const int sl[NS] = {SL_RR0, SL_RW0, SL_RS0, SL_RZ0, SL_RR, SL_K2, SL_W2, SL_T2,
                          SL_M2, SL_G2, SL_S2, SL_L2, SL_Z2, SL_Q2, SL_Y2, SL_X2,
                          SL_U2, SL_N2, SL_V2, SL_RX2, SL_RK2, SL_RL2, SL_RS2, SL_RZ2};
      double v[NS];
      if (sc->rr_auto) {
        take_sums<NS>(pre, sl, v);
      } else {
        const int sl5[5] = {SL_RR0, SL_RW0, SL_RS0, SL_RZ0, SL_RR};
        double v5[5];
        take_sums<5>(pre, sl5, v5);
        for (int d = 0; d < 5; ++d) v[d] = v5[d];
      }
      const double rho1 = v[0], rw = v[1], rs = v[2], rz = v[3], rr = v[4];
      {
        sc->sig[SL_RR0] = rho1; sc->sig[SL_RW0] = rw; sc->sig[SL_RS0] = rs;
        sc->sig[SL_RZ0] = rz; sc->sig[SL_RR] = rr;
        int its = sc->iter;
        if (mode == FIN_BETA) sc->iter = ++its;
        double* hrow = (sc->history && its >= 1 && its <= sc->hist_len)
                           ? sc->history + 4 * (int64_t)(its - 1) : nullptr;
        if (hrow) { hrow[1] = sc->alpha; hrow[2] = sc->omega; hrow[3] = 0.0; }
        if (sc->rr_auto) {
          if (mode == FIN_BETA) {
            IterNorms nm;
            nm.k = sqrt(v[5]); nm.w = sqrt(v[6]); nm.t = sqrt(v[7]); nm.m = sqrt(v[8]);
            nm.g = sqrt(v[9]); nm.s = sqrt(v[10]); nm.l = sqrt(v[11]); nm.z = sqrt(v[12]);
            nm.q = sqrt(v[13]); nm.y = sqrt(v[14]); nm.x = sqrt(v[15]); nm.u = sqrt(v[16]);
            nm.n = sqrt(v[17]); nm.v = sqrt(v[18]); nm.r = sc->rn;
            gap_bound_step(sc, sc->alpha, sc->beta, sc->omega, sc->omega_prev, nm);
          }
          if (sc->rr_hit) {
            gap_bound_reset(sc, sqrt(v[19]), sqrt(v[20]), sqrt(v[9]), sqrt(v[21]), sqrt(v[22]),
                            sqrt(v[23]));
            sc->rr_hit = 0;
          }
          if (sc->gb_prod) {
            sc->pr_its = its;     // k_bound_products logs f^r and applies eq:criterion
          } else if (sc->bound_history && its >= 1 && its <= sc->bound_len) {
            sc->bound_history[its - 1] = sc->fr;
          }
        }
        const double v5[5] = {rho1, rw, rs, rz, rr};
        // after a forced replacement the replaced residual is not tested against
        // the tolerance: the next iteration's recursive residual decides
        const G2Step g = glred2_step(v5, sc->alpha, sc->omega, sc->rho, sc->tol, sc->nb,
                                     mode == FIN_BETA);
        if (g.outcome == G2_NONFINITE) {
          stop(sc, ST_NONFINITE);
        } else {
          sc->rn = g.rn;
          if (hrow) hrow[0] = g.rn;
          if (g.outcome == G2_CONVERGED) {
            sc->done = RECURSIVE_CONVERGED;          // the host confirms with ||b - A x||
          } else {
            if (sc->rr_auto && sc->gb_prod) {        // eq:criterion, after k_bound_products
              sc->pr_rn = g.rn;
              sc->pr_op |= PR_CRIT;
            } else if (sc->rr_auto) {                // eq:criterion for the next step
              const int f_ok = sc->fr <= sc->tau * g.rn;
              sc->rr_next = sc->f_ok_prev && !f_ok;
              sc->f_ok_prev = f_ok;
            }
            if (g.outcome == G2_BREAKDOWN_OMEGA) {
              stop(sc, ST_BREAKDOWN_OMEGA);
            } else if (g.outcome == G2_BREAKDOWN_RHO) {
              stop(sc, ST_BREAKDOWN_RHO);
            } else {
              sc->beta = g.beta;
              if (hrow) hrow[3] = g.beta;
              sc->alpha = g.alpha;
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
      const double rr = pre[SL_RR];
      sc->tr = sqrt(rr);
      break;
    }
    case FIN_GAP: {
      const double rr = pre[SL_RR];
      {
        sc->gap = sqrt(rr);
        if (sc->gap_history && sc->gap_idx < sc->gap_len) sc->gap_history[sc->gap_idx] = sc->gap;
        sc->gap_idx += 1;
      }
      break;
    }
    case FIN_C_INIT: {
      // Algorithm 1 initialisation: rho_0 = (r0, r0)
      const int sl[3] = {SL_RR0, SL_RR, SL_BB};
      double v[3];
      take_sums<3>(pre, sl, v);
      const double rho = v[0], rr = v[1], bb = v[2];
      {
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
      const double sig = pre[SL_RS0];
      {
        sc->sig[SL_RS0] = sig;
        if (!finite(sig)) stop(sc, ST_NONFINITE);
        else if (sig == 0.0) stop(sc, ST_BREAKDOWN_RHO);
        else sc->alpha = sc->rho / sig;
      }
      break;
    }
    case FIN_C_BETA: {
      const int sl[2] = {SL_RR0, SL_RR};
      double v[2];
      take_sums<2>(pre, sl, v);
      const double rho1 = v[0], rr = v[1];
      {
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
    case FIN_PROBE: {
      const int sl[5] = {SL_RR0, SL_RW0, SL_RS0, SL_RZ0, SL_RR};
      double v[5];
      take_sums<5>(pre, sl, v);
      for (int d = 0; d < 5; ++d) sc->sig[sl[d]] = v[d];
      break;
    }
    case FIN_SUM: {
      const int sl[8] = {0, 1, 2, 3, 4, 5, 6, 7};
      double v[8];
      take_sums<8>(pre, sl, v);
      for (int j = 0; j < aux && j < 8; ++j) sc->sums[j] = v[j];
      break;
    }
    default:
      break;
  }
}

// A final spread over the first `fb` blocks of a kernel: block b reduces
// slots b, b + fb, ... of the mode (each with the fixed-order tree of
// block_sum_slots, so the sums are bitwise those of a one-block final),
// stores them, and arrives at a counter; the last block to arrive runs the
// scalar logic on the stored sums.  No block waits for another.  Inlined
// into each caller: compiled as one shared function it took 184 VGPRs, and a
// kernel's count includes its callees', which left every SPMV at two waves
// per SIMD; inlined, the SPMVs need 108 (four waves).
__device__ __forceinline__ void distributed_final(int mode, DevScalars* __restrict__ sc,
                                                  const double* __restrict__ partials, int nblk,
                                                  int fb, int rr_auto) {
  const FinSlots fs = fin_slots(mode, rr_auto, 0);
  for (int d = blockIdx.x; d < fs.n; d += fb) {
    const int slot = fs.s[d];
    const double v = block_sum_slot(partials, slot, nblk);
    if (threadIdx.x == 0)
      __hip_atomic_store(&sc->red[slot], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __shared__ int last;
  if (threadIdx.x == 0) {
    const int old = __hip_atomic_fetch_add(&sc->fin_arrive, 1, __ATOMIC_ACQ_REL,
                                           __HIP_MEMORY_SCOPE_AGENT);
    last = old == fb - 1;
  }
  __syncthreads();
  if (!last) return;
  // every slot block has arrived: the struct (red[] included) is complete
  __shared__ DevScalars lsc;
  scalars_to_lds(sc, &lsc);
  if (threadIdx.x == 0) {
    lsc.fin_arrive = 0;
    run_final(mode, &lsc, lsc.red, 0);
  }
  scalars_from_lds(sc, &lsc);
}

// A final in one block: the scalar struct and the partials of all the
// mode's slots are loaded together (one memory round trip), reduced with the
// fixed-order tree of block_sum_slots, and one thread runs the scalar logic
// on an LDS copy of the struct.  NS >= fs.n; the slots past fs.n repeat the
// first one and are not used.
template <int NS>
__device__ inline void one_block_final(int mode, const FinSlots& fs, DevScalars* __restrict__ sc,
                                       const double* __restrict__ partials, int nblk, int aux,
                                       bool respect_done) {
  static_assert(kScWords <= 2 * kBlock, "two struct words per thread at most");
  __shared__ DevScalars lsc;
  __shared__ double pre[kNumSlots];
  const uint32_t* src = reinterpret_cast<const uint32_t*>(sc);
  const int tid = threadIdx.x;
  uint32_t w0 = 0, w1 = 0;
  if (tid < kScWords) w0 = __hip_atomic_load(src + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (tid + kBlock < kScWords)
    w1 = __hip_atomic_load(src + tid + kBlock, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  int sl[NS];
#pragma unroll
  for (int d = 0; d < NS; ++d) sl[d] = d < fs.n ? fs.s[d] : fs.s[0];
  double v[NS];
  block_sum_slots<NS>(partials, sl, nblk, v);
  uint32_t* dst = reinterpret_cast<uint32_t*>(&lsc);
  if (tid < kScWords) dst[tid] = w0;
  if (tid + kBlock < kScWords) dst[tid + kBlock] = w1;
  if (tid == 0) {
#pragma unroll
    for (int d = 0; d < NS; ++d)            // compile-time indices keep v[] in registers
      if (d < fs.n) pre[sl[d]] = v[d];
  }
  __syncthreads();
  if (respect_done && lsc.done) return;
  if (tid == 0) run_final(mode, &lsc, pre, aux);
  scalars_from_lds(sc, &lsc);
}

}  // namespace pbcg
