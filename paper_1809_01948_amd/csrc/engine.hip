// Host engine of the pipelined BiCGStab library: layouts, the solve loops
// and the exported C ABI (include/pbicgstab.h).
//
// Iteration schedule of Algorithm 2 on one GPU (one stream, 4 kernels per
// iteration, no host synchronisation inside the loop):
//   phaseA   g, s, l, z recurrences; partials (q,y), (y,y)           [GLRED 1 begins]
//   spmv     v = A M^-1 z; its block 0 reduces GLRED 1 -> omega_i    [GLRED 1 ends]
//   phaseB   x, r, k, w recurrences; partials of GLRED 2             [GLRED 2 begins]
//   (rr1, rr2: residual replacement, predicated on the device)
//   spmv     t = A M^-1 w; its block 0 reduces GLRED 2 -> beta, alpha [GLRED 2 ends]
// All scalars stay on the device.  The host launches chunks of iterations
// and reads the device status block (pinned copy) one chunk behind, so the
// GPU never waits for the host; kernels of an already finished solve exit at
// their first instruction.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pbicgstab.h"
#include "solver.hpp"

namespace pbcg {
void launch_dia5_transpose(Solver& S, hipStream_t st);
}

using namespace pbcg;

struct pbcg_solver {
  Solver S;
};

namespace {

thread_local std::string g_last_error;

struct PbcgError : std::runtime_error {
  int code;
  PbcgError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(int code, const std::string& msg) { throw PbcgError(code, msg); }

void hipck(hipError_t e, const char* what) {
  if (e != hipSuccess)
    fail(PBCG_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <class F>
int guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const PbcgError& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return PBCG_ERR_HIP;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return PBCG_ERR_INVALID_ARG;
  }
}

int64_t round_up(int64_t a, int64_t m) { return (a + m - 1) / m * m; }

// Device memory of a handle: consecutive 256-byte aligned pieces of the
// caller's workspace, zeroed.  The pieces and their order are those that
// pbicgstab_workspace_bytes adds up (layout_bytes).
void* dalloc(Solver& S, size_t bytes) {
  if (bytes == 0) bytes = 256;
  const size_t off = (size_t)round_up((int64_t)S.ws_used, kWsAlign);
  if (off + bytes > S.ws_size)
    fail(PBCG_ERR_WORKSPACE_TOO_SMALL,
         "workspace too small: " + std::to_string(off + bytes) + " bytes needed so far, " +
             std::to_string(S.ws_size) + " given (size it with pbicgstab_workspace_bytes)");
  void* p = S.ws + off;
  S.ws_used = off + bytes;
  hipck(hipMemset(p, 0, bytes), "hipMemset");
  return p;
}

// Block size encoded in a precond argument (PBCG_PC_BLOCK_JACOBI(b)), else 0.
int64_t block_size_of(int precond) {
  if ((precond & ~0xff) != PBCG_PC_BLOCK_JACOBI_BASE) return 0;
  const int b = precond & 0xff;
  return (b >= 2 && b <= 64) ? b : 0;
}

// Workspace bytes of one layout (see pbicgstab_workspace_bytes): the same
// pieces, in the same order and alignment, as create and the transpose build
// take.  For sliced ELL, `width` bounds every slice's width (the longest row,
// and for the transpose the longest column).
size_t layout_bytes(int format, int64_t n, int64_t nnz, int64_t width, int precision,
                    int precond, bool with_transpose) {
  const int64_t ts = precision == PBCG_FP64 ? 8 : 4;
  const int64_t npad = round_up(n, kPadElems);
  int64_t used = 0;
  auto take = [&](int64_t bytes) {
    if (bytes == 0) bytes = 256;
    used = round_up(used, kWsAlign) + bytes;
  };
  for (int v = 0; v < V_COUNT; ++v) take(npad * ts);
  take(npad * 8);                                   // x
  take(npad * 8);                                   // b
  take((int64_t)sizeof(double) * kNumSlots * kMaxPartials);
  take(2 * (int64_t)sizeof(DevScalars));
  const int64_t block = block_size_of(precond);
  if (format == PBCG_CSR && block > 0) {
    // A M^-1 (each stored entry spreads over one block of columns), then
    // M and M^-1 in FP64 and the FP64 scratch vector
    const int64_t ns = (n + kSellC - 1) / kSellC;
    const int64_t wt = std::min<int64_t>(n, width * block);
    const int64_t nlb = (n + kLdsRows - 1) / kLdsRows;
    take((ns + 1) * 8);
    take(ns * kSellC * wt * 4);
    take(ns * kSellC * wt * ts);
    take(nlb * 4);
    take(nlb * 4);
    for (int k = 0; k < 2; ++k) {
      take((ns + 1) * 8);
      take(ns * kSellC * block * 4);
      take(ns * kSellC * block * 8);
    }
    take(npad * 8);
    return (size_t)round_up(used, kWsAlign);
  }
  if (format == PBCG_CSR) {
    const int64_t ns = (n + kSellC - 1) / kSellC;
    const int64_t elems = ns * kSellC * width;
    const int64_t nlb = (n + kLdsRows - 1) / kLdsRows;
    auto sell = [&]() {
      take((ns + 1) * 8);
      take(elems * 4);
      take(elems * ts);
      take(nlb * 4);                                // LDS windows: first column
      take(nlb * 4);                                //   and length
    };
    sell();                                         // A
    take(std::max<int64_t>(nnz, 1) * 8);            // CSR entry -> SELL slot
    take((n + 1) * 4);                              // rowptr
    take(std::max<int64_t>(nnz, 1) * 4);            // col
    take(n * 8);                                    // diagonal positions
    if (precond) take(npad * ts);                   // dinv
    if (with_transpose) {
      sell();                                       // A^T
      take(std::max<int64_t>(nnz, 1) * 8);
    }
  } else if (format == PBCG_ST_DIA5) {
    take(5 * npad * ts);
    if (precond) take(npad * ts);
    if (with_transpose) take(5 * npad * ts);
  }
  return (size_t)round_up(used, kWsAlign);
}

// A recursive convergence whose FP64 true residual misses the tolerance is
// followed by a replacement and more iterations at most this many times per
// solve; the next such failure ends it with TRUE_RES_NOT_MET.
constexpr int kMaxForcedReplacements = 3;

void common_setup(Solver& S, int precision, int precond, void* workspace, size_t ws_bytes) {
  if (!workspace) fail(PBCG_ERR_INVALID_ARG, "workspace is null");
  if (((uintptr_t)workspace) % kWsAlign != 0)
    fail(PBCG_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  S.ws = (char*)workspace;
  S.ws_size = ws_bytes;
  S.ws_used = 0;
  if (precision != PBCG_FP64 && precision != PBCG_MIXED) fail(PBCG_ERR_INVALID_ARG, "precision must be PBCG_FP64 or PBCG_MIXED");
  if (precond != PBCG_PC_NONE && precond != PBCG_PC_JACOBI)
    fail(PBCG_ERR_INVALID_ARG, "precond must be PBCG_PC_NONE, PBCG_PC_JACOBI or (CSR only) "
                               "PBCG_PC_BLOCK_JACOBI(b) with 2 <= b <= 64");
  if (S.n > (int64_t)2000000000) fail(PBCG_ERR_UNSUPPORTED, "n exceeds the int32 index range");
  S.precision = precision;
  S.precond = precond;
  S.tsize = precision == PBCG_FP64 ? 8 : 4;
  S.npad = round_up(S.n, kPadElems);
  const int vw = (int)(16 / S.tsize);
  S.vtiles = S.npad / (kBlock * vw);
  S.rtiles = (S.n + kBlock - 1) / kBlock;
  // Streaming kernels: at most 1024 blocks, so that every block of a phase
  // kernel (70-96 VGPRs, 4-7 resident blocks per CU) is resident at once and
  // loops over its tiles, with no second wave of blocks at the tail
  // (measured: 1000^2 Poisson iteration 52.1 -> 49.3 us, unchanged at 200^3).
  // The SpMVs keep up to 2048 work blocks.
  const int64_t tiles = std::max<int64_t>(S.vtiles, S.rtiles);
  int64_t nb = std::min<int64_t>(kMaxPartials, tiles);
  if (const char* env = std::getenv("PBCG_NBLK")) {   // tuning override
    const long v = std::strtol(env, nullptr, 10);
    if (v > 0) nb = v;
  }
  nb = round_up(std::max<int64_t>(nb, kXcds), kXcds);
  if (nb > kMaxPartials) nb = kMaxPartials;
  S.nblk = (int)nb;
  S.nspmv = (int)std::min<int64_t>(kMaxBlocks, round_up(std::max<int64_t>(tiles, kXcds), kXcds));
  if (const char* env = std::getenv("PBCG_SPMV_BLOCKS")) {   // tuning override
    const long v = std::strtol(env, nullptr, 10);
    if (v > 0) S.nspmv = (int)std::min<long>(kMaxBlocks, round_up(std::max<long>(v, kXcds), kXcds));
  }
  // Non-temporal streaming pays once the solver's vectors no longer fit the
  // 256 MB Infinity Cache (measured: phase B on 8e6 FP64 rows 190 -> 144 us);
  // below that it costs a little.  Mixed-precision phase A is faster with
  // cached accesses at every size measured.
  const int64_t footprint = (int64_t)(V_COUNT * S.tsize + 16) * S.npad;
  if (footprint > ((int64_t)192 << 20)) S.vnt = precision == PBCG_FP64 ? 3 : 2;
  if (const char* env = std::getenv("PBCG_VEC_NT")) S.vnt = std::atoi(env) & 3;
  if (const char* env = std::getenv("PBCG_SPMV_TILED")) S.spmv_tiled = std::atoi(env) != 0;
  if (const char* env = std::getenv("PBCG_FUSE")) S.fuse = std::atoi(env) != 0;
  if (const char* env = std::getenv("PBCG_MARCH3D")) S.march3d = std::atoi(env) != 0;
  if (const char* env = std::getenv("PBCG_MARCH_PHASE")) S.march_phase = std::atoi(env) != 0;
  if (const char* env = std::getenv("PBCG_PREMULT")) S.premult = std::atoi(env) != 0;
  if (const char* env = std::getenv("PBCG_SELL_LDS")) S.sell_lds = std::atoi(env) != 0;
  if (const char* env = std::getenv("PBCG_LDS_BLOCKS")) S.lds_blocks = std::atoi(env);
  if (const char* env = std::getenv("PBCG_SMALL_RPT")) {
    const int v = std::atoi(env);
    S.small_rpt = (v == 1 || v == 4) ? v : 2;
  }
  {
    int dev = 0, cap = 0;
    hipck(hipGetDevice(&dev), "hipGetDevice");
    hipck(hipDeviceGetAttribute(&cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev),
          "hipDeviceGetAttribute");
    S.lds_cap = cap;
  }
  if (const char* env = std::getenv("PBCG_MARCH_ZLEN")) S.march_zlen = std::atoi(env);
  hipck(hipStreamCreateWithFlags(&S.s1, hipStreamNonBlocking), "hipStreamCreate");
  hipck(hipEventCreateWithFlags(&S.ev_in, hipEventDisableTiming), "hipEventCreate");
  hipck(hipEventCreateWithFlags(&S.ev_out, hipEventDisableTiming), "hipEventCreate");
  hipck(hipEventCreateWithFlags(&S.ev_poll[0], hipEventDisableTiming), "hipEventCreate");
  hipck(hipEventCreateWithFlags(&S.ev_poll[1], hipEventDisableTiming), "hipEventCreate");
  hipck(hipEventCreate(&S.ev_t0), "hipEventCreate");
  hipck(hipEventCreate(&S.ev_t1), "hipEventCreate");
  for (int v = 0; v < V_COUNT; ++v) S.vec[v] = dalloc(S, S.npad * S.tsize);
  S.x = (double*)dalloc(S, S.npad * 8);
  S.b = (double*)dalloc(S, S.npad * 8);
  S.partials = (double*)dalloc(S, sizeof(double) * kNumSlots * kMaxPartials);
  S.sc = (DevScalars*)dalloc(S, 2 * sizeof(DevScalars));
  hipck(hipHostMalloc((void**)&S.h_sc, 3 * sizeof(DevScalars), hipHostMallocDefault),
        "hipHostMalloc");
  std::memset(S.h_sc, 0, 3 * sizeof(DevScalars));
}

// CSR -> SELL-64 on the host; pos[k] = SELL slot of CSR entry k
void build_sell(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                std::vector<int64_t>& sptr, std::vector<int32_t>& scol, std::vector<double>& sval,
                std::vector<int64_t>& pos, int& max_width) {
  const int64_t ns = (n + kSellC - 1) / kSellC;
  sptr.assign(ns + 1, 0);
  max_width = 0;
  for (int64_t s = 0; s < ns; ++s) {
    int w = 0;
    for (int64_t i = s * kSellC; i < std::min<int64_t>(n, (s + 1) * kSellC); ++i)
      w = std::max<int>(w, rowptr[i + 1] - rowptr[i]);
    max_width = std::max(max_width, w);
    sptr[s + 1] = sptr[s] + (int64_t)w * kSellC;
  }
  scol.assign(sptr[ns], -1);
  sval.assign(sptr[ns], 0.0);
  pos.assign(rowptr[n], 0);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t s = i / kSellC, lane = i % kSellC;
    int j = 0;
    for (int64_t kk = rowptr[i]; kk < rowptr[i + 1]; ++kk, ++j) {
      const int64_t p = sptr[s] + (int64_t)j * kSellC + lane;
      scol[p] = col[kk];
      sval[p] = val[kk];
      pos[kk] = p;
    }
  }
}

template <typename T>
void upload_vals(Solver& S, void* dst, const std::vector<double>& v) {
  std::vector<T> t(v.size());
  for (size_t i = 0; i < v.size(); ++i) t[i] = (T)v[i];
  hipck(hipMemcpy(dst, t.data(), t.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
}

void upload_sell(Solver& S, OpData& o, const std::vector<int64_t>& sptr,
                 const std::vector<int32_t>& scol, const std::vector<double>& sval, int mw,
                 bool fp64 = false) {
  o.kind = OP_SELL;
  o.nslices = (int64_t)sptr.size() - 1;
  o.sell_elems = sptr.back();
  o.max_width = mw;
  o.sptr = (int64_t*)dalloc(S, sptr.size() * 8);
  o.col = (int32_t*)dalloc(S, scol.size() * 4);
  o.val = dalloc(S, sval.size() * (fp64 ? 8 : S.tsize));
  hipck(hipMemcpy(o.sptr, sptr.data(), sptr.size() * 8, hipMemcpyHostToDevice), "hipMemcpy");
  hipck(hipMemcpy(o.col, scol.data(), scol.size() * 4, hipMemcpyHostToDevice), "hipMemcpy");
  if (fp64 || S.precision == PBCG_FP64) upload_vals<double>(S, o.val, sval);
  else upload_vals<float>(S, o.val, sval);
  if (fp64) return;
  // column window of each block of kLdsRows rows: the columns its entries
  // read and the rows themselves (a padding entry reads its own row)
  const int64_t n = S.n, nlb = (n + kLdsRows - 1) / kLdsRows;
  std::vector<int32_t> wlo(nlb), wlen(nlb);
  int wmax = 0;
  for (int64_t t = 0; t < nlb; ++t) {
    int64_t lo = t * kLdsRows, hi = std::min<int64_t>(n, lo + kLdsRows) - 1;
    const int64_t s0 = t * (kLdsRows / kSellC);
    const int64_t s1 = std::min<int64_t>(o.nslices, s0 + kLdsRows / kSellC);
    for (int64_t e = sptr[s0]; e < sptr[s1]; ++e)
      if (scol[e] >= 0) {
        lo = std::min<int64_t>(lo, scol[e]);
        hi = std::max<int64_t>(hi, scol[e]);
      }
    wlo[t] = (int32_t)lo;
    wlen[t] = (int32_t)(hi - lo + 1);
    wmax = std::max(wmax, wlen[t]);
  }
  o.nlb = nlb;
  o.win_max = wmax;
  o.win_lo = (int32_t*)dalloc(S, nlb * 4);
  o.win_len = (int32_t*)dalloc(S, nlb * 4);
  hipck(hipMemcpy(o.win_lo, wlo.data(), nlb * 4, hipMemcpyHostToDevice), "hipMemcpy");
  hipck(hipMemcpy(o.win_len, wlen.data(), nlb * 4, hipMemcpyHostToDevice), "hipMemcpy");
}

// Jacobi diagonal (sum of the entries with col == row) from the host CSR
void set_dinv_csr(Solver& S) {
  std::vector<double> d(S.npad, 0.0);
  std::vector<int64_t> dpos(S.n, -1);
  for (int64_t i = 0; i < S.n; ++i) {
    double s = 0.0;
    for (int64_t kk = S.h_rowptr[i]; kk < S.h_rowptr[i + 1]; ++kk)
      if (S.h_col[kk] == i) {
        s += S.h_val[kk];
        if (dpos[i] < 0) dpos[i] = kk;
      }
    d[i] = s;
  }
  S.d_diagpos = (int64_t*)dalloc(S, S.n * 8);
  hipck(hipMemcpy(S.d_diagpos, dpos.data(), S.n * 8, hipMemcpyHostToDevice), "hipMemcpy");
  if (!S.precond) return;
  S.pc = PC_VECTOR;
  S.dinv = dalloc(S, S.npad * S.tsize);
  if (S.precision == PBCG_FP64) {
    std::vector<double> di(S.npad, 0.0);
    for (int64_t i = 0; i < S.n; ++i) {
      if (d[i] == 0.0) fail(PBCG_ERR_ZERO_DIAG, "zero diagonal entry in row " + std::to_string(i));
      di[i] = 1.0 / d[i];
    }
    hipck(hipMemcpy(S.dinv, di.data(), S.npad * 8, hipMemcpyHostToDevice), "hipMemcpy");
  } else {
    std::vector<float> di(S.npad, 0.0f);
    for (int64_t i = 0; i < S.n; ++i) {
      const float df = (float)d[i];
      if (df == 0.0f) fail(PBCG_ERR_ZERO_DIAG, "zero diagonal entry in row " + std::to_string(i));
      di[i] = 1.0f / df;
    }
    hipck(hipMemcpy(S.dinv, di.data(), S.npad * 4, hipMemcpyHostToDevice), "hipMemcpy");
  }
}

// ||A||_2 <= sqrt(||A||_1 ||A||_inf) and the maximum stored entries per row
// and per column, from host data (the automated replacement bound).
void set_norm_bounds(Solver& S, const std::vector<double>& rowsum,
                     const std::vector<double>& colsum, int mu_row, int mu_col) {
  double r = 0.0, c = 0.0;
  for (double v : rowsum) r = std::max(r, v);
  for (double v : colsum) c = std::max(c, v);
  S.normA = std::sqrt(c * r);
  S.mu_row = mu_row;
  S.mu_col = mu_col;
}

void norms_csr(Solver& S) {
  std::vector<double> rs(S.n, 0.0), cs(S.n, 0.0);
  std::vector<int> cc(S.n, 0);
  int mr = 0;
  for (int64_t i = 0; i < S.n; ++i) {
    mr = std::max<int>(mr, S.h_rowptr[i + 1] - S.h_rowptr[i]);
    for (int64_t kk = S.h_rowptr[i]; kk < S.h_rowptr[i + 1]; ++kk) {
      rs[i] += std::fabs(S.h_val[kk]);
      cs[S.h_col[kk]] += std::fabs(S.h_val[kk]);
      cc[S.h_col[kk]] += 1;
    }
  }
  int mc = 0;
  for (int v : cc) mc = std::max(mc, v);
  set_norm_bounds(S, rs, cs, mr, mc);
}

// constant stencils and DIA5: row and column sums over the actual grid
void norms_grid(Solver& S, const double* dia /* 5*n or null */) {
  const OpData& o = S.A;
  const int nd = S.kind == OP_ST3D7 ? 7 : 5;
  const int64_t nx = o.dims[0], ny = o.dims[1], nz = S.kind == OP_ST3D7 ? o.dims[2] : 1;
  const int64_t off[7] = {-nx * ny, -nx, -1, 0, 1, nx, nx * ny};
  const int base = nd == 7 ? 0 : 1;   // 2D uses off[1..5]
  std::vector<double> rs(S.n, 0.0), cs(S.n, 0.0);
  int mr = 0;
  for (int64_t p = 0; p < S.n; ++p) {
    const int64_t iz = p / (nx * ny), rem = p % (nx * ny), iy = rem / nx, ix = rem % nx;
    const bool has[7] = {iz > 0, iy > 0, ix > 0, true, ix < nx - 1, iy < ny - 1, iz < nz - 1};
    int cnt = 0;
    for (int d = 0; d < nd; ++d) {
      const int dd = base + d;
      if (!has[dd]) continue;
      const double a = dia ? dia[d * S.n + p] : o.c64[d];
      rs[p] += std::fabs(a);
      cs[p + off[dd]] += std::fabs(a);
      ++cnt;
    }
    mr = std::max(mr, cnt);
  }
  set_norm_bounds(S, rs, cs, mr, mr);
}

// Block-Jacobi set-up on the host from the input CSR (rowptr, col, val):
// the diagonal blocks of `bs` consecutive rows and columns (the last one
// ragged) are inverted by Gauss-Jordan elimination with partial pivoting; the
// operator stored for the iteration is A M^-1 (row i: every stored a_ij
// spread over the columns of j's block with the weights of row j of M^-1,
// summed per column in ascending order), and M, M^-1 are stored as FP64
// sliced ELL.  Right preconditioning then needs no PREC step inside the
// iteration: Algorithm 2 on A M^-1 with y_0 = M x_0 gives the same residuals,
// scalars and x_i = M^-1 y_i in exact arithmetic.
void setup_block_jacobi(Solver& S, int bs, std::vector<int32_t>& rowptr, std::vector<int32_t>& col,
                        std::vector<double>& val) {
  const int64_t n = S.n, nblk = (n + bs - 1) / bs;
  std::vector<double> inv((size_t)nblk * bs * bs, 0.0), mblk((size_t)nblk * bs * bs, 0.0);
  std::vector<double> a((size_t)bs * 2 * bs);
  for (int64_t blk = 0; blk < nblk; ++blk) {
    const int64_t lo = blk * bs, m = std::min<int64_t>(bs, n - lo);
    double* M = &mblk[(size_t)blk * bs * bs];
    for (int64_t r = 0; r < m; ++r)
      for (int64_t kk = rowptr[lo + r]; kk < rowptr[lo + r + 1]; ++kk)
        if (col[kk] >= lo && col[kk] < lo + m) M[r * bs + (col[kk] - lo)] += val[kk];
    // [M | I] -> [I | M^-1]
    for (int64_t r = 0; r < m; ++r)
      for (int64_t c = 0; c < 2 * m; ++c)
        a[r * 2 * bs + c] = c < m ? M[r * bs + c] : (c - m == r ? 1.0 : 0.0);
    for (int64_t c = 0; c < m; ++c) {
      int64_t piv = c;
      for (int64_t r = c + 1; r < m; ++r)
        if (std::fabs(a[r * 2 * bs + c]) > std::fabs(a[piv * 2 * bs + c])) piv = r;
      if (a[piv * 2 * bs + c] == 0.0)
        fail(PBCG_ERR_ZERO_DIAG, "singular diagonal block at rows " + std::to_string(lo) + ".." +
                                     std::to_string(lo + m - 1));
      if (piv != c)
        for (int64_t k = 0; k < 2 * m; ++k) std::swap(a[c * 2 * bs + k], a[piv * 2 * bs + k]);
      const double d = a[c * 2 * bs + c];
      for (int64_t k = 0; k < 2 * m; ++k) a[c * 2 * bs + k] /= d;
      for (int64_t r = 0; r < m; ++r) {
        if (r == c) continue;
        const double f = a[r * 2 * bs + c];
        if (f == 0.0) continue;
        for (int64_t k = 0; k < 2 * m; ++k) a[r * 2 * bs + k] -= f * a[c * 2 * bs + k];
      }
    }
    double* I = &inv[(size_t)blk * bs * bs];
    for (int64_t r = 0; r < m; ++r)
      for (int64_t c = 0; c < m; ++c) I[r * bs + c] = a[r * 2 * bs + m + c];
  }
  // A M^-1
  std::vector<int32_t> trp(n + 1, 0), tcol;
  std::vector<double> tval;
  std::vector<double> acc(n, 0.0);
  std::vector<int32_t> touched;
  std::vector<char> seen(n, 0);
  for (int64_t i = 0; i < n; ++i) {
    touched.clear();
    for (int64_t kk = rowptr[i]; kk < rowptr[i + 1]; ++kk) {
      const int64_t j = col[kk], blk = j / bs, lo = blk * bs, m = std::min<int64_t>(bs, n - lo);
      const double* I = &inv[(size_t)blk * bs * bs + (size_t)(j - lo) * bs];
      for (int64_t c = 0; c < m; ++c) {
        if (!seen[lo + c]) {
          seen[lo + c] = 1;
          touched.push_back((int32_t)(lo + c));
        }
        acc[lo + c] += val[kk] * I[c];
      }
    }
    std::sort(touched.begin(), touched.end());
    for (int32_t c : touched) {
      tcol.push_back(c);
      tval.push_back(acc[c]);
      acc[c] = 0.0;
      seen[c] = 0;
    }
    trp[i + 1] = (int32_t)tcol.size();
  }
  // M and M^-1 as sliced ELL (row i: the columns of its block)
  auto block_sell = [&](const std::vector<double>& src, OpData& o) {
    std::vector<int32_t> brp(n + 1, 0), bcol;
    std::vector<double> bval;
    for (int64_t i = 0; i < n; ++i) {
      const int64_t blk = i / bs, lo = blk * bs, m = std::min<int64_t>(bs, n - lo);
      for (int64_t c = 0; c < m; ++c) {
        bcol.push_back((int32_t)(lo + c));
        bval.push_back(src[(size_t)blk * bs * bs + (size_t)(i - lo) * bs + c]);
      }
      brp[i + 1] = (int32_t)bcol.size();
    }
    std::vector<int64_t> sptr, pos;
    std::vector<int32_t> scol;
    std::vector<double> sval;
    int mw = 0;
    build_sell(n, brp.data(), bcol.data(), bval.data(), sptr, scol, sval, pos, mw);
    upload_sell(S, o, sptr, scol, sval, mw, true);
  };
  {
    std::vector<int64_t> sptr, pos;
    std::vector<int32_t> scol;
    std::vector<double> sval;
    int mw = 0;
    build_sell(n, trp.data(), tcol.data(), tval.data(), sptr, scol, sval, pos, mw);
    upload_sell(S, S.A, sptr, scol, sval, mw);
  }
  block_sell(mblk, S.Mb);
  block_sell(inv, S.Bi);
  S.ytmp = (double*)dalloc(S, S.npad * 8);
  rowptr = std::move(trp);
  col = std::move(tcol);
  val = std::move(tval);
  S.nnz = (int64_t)col.size();
  S.block = bs;
}

// Values of the host CSR copy into a sliced-ELL layout whose slot of CSR
// entry k is pos[k] (padding slots stay 0).
void upload_scattered(Solver& S, OpData& o, const std::vector<int64_t>& pos) {
  std::vector<double> sval(o.sell_elems, 0.0);
  for (int64_t kk = 0; kk < S.nnz; ++kk) sval[pos[kk]] = S.h_val[kk];
  if (S.precision == PBCG_FP64) upload_vals<double>(S, o.val, sval);
  else upload_vals<float>(S, o.val, sval);
}

// Jacobi diagonal (sum of the entries with col == row) of the host CSR copy
void upload_dinv_csr(Solver& S) {
  std::vector<double> di(S.npad, 0.0);
  for (int64_t i = 0; i < S.n; ++i) {
    double d = 0.0;
    for (int64_t kk = S.h_rowptr[i]; kk < S.h_rowptr[i + 1]; ++kk)
      if (S.h_col[kk] == i) d += S.h_val[kk];
    if (S.precision == PBCG_FP64) {
      if (d == 0.0) fail(PBCG_ERR_ZERO_DIAG, "zero diagonal after value update");
      di[i] = 1.0 / d;
    } else {
      if ((float)d == 0.0f) fail(PBCG_ERR_ZERO_DIAG, "zero diagonal after value update");
      di[i] = (double)(1.0f / (float)d);
    }
  }
  if (S.precision == PBCG_FP64) upload_vals<double>(S, S.dinv, di);
  else upload_vals<float>(S, S.dinv, di);
}

// After the DIA5 coefficients changed on the device: the host copy and the
// bounds of the automated criterion (||A|| from the row and column sums,
// ||M^-1|| = max |1 / a_ii|) from the stored coefficients.
void refresh_dia5_bounds(Solver& S) {
  const int64_t n = S.n;
  std::vector<double> host(5 * n);
  if (S.precision == PBCG_FP64) {
    std::vector<double> t(5 * S.npad);
    hipck(hipMemcpy(t.data(), S.A.dia, t.size() * 8, hipMemcpyDeviceToHost), "hipMemcpy");
    for (int d = 0; d < 5; ++d)
      for (int64_t i = 0; i < n; ++i) host[d * n + i] = t[d * S.npad + i];
  } else {
    std::vector<float> t(5 * S.npad);
    hipck(hipMemcpy(t.data(), S.A.dia, t.size() * 4, hipMemcpyDeviceToHost), "hipMemcpy");
    for (int d = 0; d < 5; ++d)
      for (int64_t i = 0; i < n; ++i) host[d * n + i] = (double)t[d * S.npad + i];
  }
  S.h_dia = std::move(host);
  norms_grid(S, S.h_dia.data());
  if (S.precond) {
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) m = std::max(m, std::fabs(1.0 / S.h_dia[2 * n + i]));
    S.normM = m;
  }
}

void build_transpose(Solver& S) {
  if (S.have_AT) return;
  if (S.kind == OP_SELL) {
    const int64_t n = S.n, nnz = S.nnz;
    std::vector<int32_t> trp(n + 1, 0), tcol(nnz);
    std::vector<double> tval(nnz);
    std::vector<int64_t> where(nnz);  // CSR entry -> position in the transposed CSR
    for (int64_t kk = 0; kk < nnz; ++kk) trp[S.h_col[kk] + 1]++;
    for (int64_t i = 0; i < n; ++i) trp[i + 1] += trp[i];
    std::vector<int32_t> fillp(trp.begin(), trp.end() - 1);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t kk = S.h_rowptr[i]; kk < S.h_rowptr[i + 1]; ++kk) {
        const int32_t j = S.h_col[kk];
        const int64_t q = fillp[j]++;
        tcol[q] = (int32_t)i;
        tval[q] = S.h_val[kk];
        where[kk] = q;
      }
    std::vector<int64_t> sptr, pos;
    std::vector<int32_t> scol;
    std::vector<double> sval;
    int mw = 0;
    build_sell(n, trp.data(), tcol.data(), tval.data(), sptr, scol, sval, pos, mw);
    upload_sell(S, S.AT, sptr, scol, sval, mw);
    S.h_posAT.assign(nnz, 0);
    for (int64_t kk = 0; kk < nnz; ++kk) S.h_posAT[kk] = pos[where[kk]];
    S.d_posAT = (int64_t*)dalloc(S, std::max<int64_t>(nnz, 1) * 8);
    hipck(hipMemcpy(S.d_posAT, S.h_posAT.data(), nnz * 8, hipMemcpyHostToDevice), "hipMemcpy");
  } else if (S.kind == OP_ST2D5 || S.kind == OP_ST3D7) {
    S.AT = S.A;
    const int nd = S.kind == OP_ST2D5 ? 5 : 7;
    for (int d = 0; d < nd; ++d) {
      S.AT.c64[d] = S.A.c64[nd - 1 - d];
      S.AT.c32[d] = S.A.c32[nd - 1 - d];
    }
  } else {
    S.AT = S.A;
    S.AT.dia = dalloc(S, 5 * S.npad * S.tsize);
    launch_dia5_transpose(S, S.s1);
    hipck(hipGetLastError(), "dia5 transpose launch");
    hipck(hipStreamSynchronize(S.s1), "hipStreamSynchronize");
  }
  S.have_AT = true;
}

DevScalars initial_scalars(const Solver& S, const pbcg_opts& o, bool tr) {
  DevScalars d;
  std::memset(&d, 0, sizeof(d));
  d.tol = o.tol;
  d.tau = o.rr_tau > 0 ? o.rr_tau : std::sqrt(std::ldexp(1.0, -53));
  d.bound_history = o.bound_history;
  d.bound_len = o.bound_history ? o.bound_len : 0;
  d.rr_auto = o.rr_auto ? 1 : 0;
  d.rr_est = (o.rr_auto == 2 || o.rr_auto == 4) ? 1 : 0;
  d.gb_prod = o.rr_auto >= 3 ? 1 : 0;
  d.pr_state = o.rr_auto >= 3 ? o.bound_state : nullptr;
  d.pr_cap = o.rr_auto >= 3 ? o.bound_state_len / kBoundStateArrays : 0;
  d.eps_b = o.rr_eps > 0 ? o.rr_eps : std::ldexp(1.0, S.precision == PBCG_FP64 ? -53 : -24);
  d.eps_r = std::ldexp(1.0, -53);     // replacements are computed in FP64
  if (o.rr_auto && !(o.rr_tau > 0)) d.tau = std::sqrt(d.eps_b);
  d.nA = S.normA;
  d.nM = S.normM;
  d.mu = tr ? S.mu_col : S.mu_row;
  d.nN = (double)S.n;
  d.maxit = o.maxit;
  d.rr_period = o.rr_period;
  d.history = o.history;
  d.hist_len = o.history ? o.history_len : 0;
  d.gap_history = o.gap_history;
  d.gap_len = o.gap_history ? o.gap_len : 0;
  return d;
}

void validate_opts(const pbcg_opts& o) {
  if (!(o.tol >= 0.0)) fail(PBCG_ERR_INVALID_ARG, "tol must be >= 0");
  if (o.maxit < 1) fail(PBCG_ERR_INVALID_ARG, "maxit must be >= 1");
  if (o.rr_period < 0) fail(PBCG_ERR_INVALID_ARG, "rr_period must be >= 0");
  if (o.rr_tau < 0) fail(PBCG_ERR_INVALID_ARG, "rr_tau must be >= 0");
  if (o.check_every < 0) fail(PBCG_ERR_INVALID_ARG, "check_every must be >= 0");
  if (o.history_len < 0 || o.gap_len < 0 || o.gap_every < 0 || o.bound_len < 0)
    fail(PBCG_ERR_INVALID_ARG, "negative history length");
  if (o.rr_auto < 0 || o.rr_auto > 4) fail(PBCG_ERR_INVALID_ARG, "rr_auto must be 0 .. 4");
  if (o.rr_auto >= 3 &&
      (!o.bound_state || o.bound_state_len < kBoundStateArrays * ((int64_t)o.maxit + 2)))
    fail(PBCG_ERR_INVALID_ARG, "rr_auto 3 or 4 needs bound_state of at least 16 * (maxit + 2) "
                               "doubles");
}

// Upload scalars, copy b and x0 into the padded internal vectors.
void begin_solve(Solver& S, const double* b, const double* x, const pbcg_opts& o,
                 hipStream_t cs) {
  if (!b || !x) fail(PBCG_ERR_INVALID_ARG, "b and x must be device pointers");
  hipck(hipEventRecord(S.ev_in, cs), "hipEventRecord");
  hipck(hipStreamWaitEvent(S.s1, S.ev_in, 0), "hipStreamWaitEvent");
  S.rhat_in = o.rhat;
  S.h_sc[2] = initial_scalars(S, o, o.transpose != 0);
  hipck(hipMemcpyAsync(S.sc, &S.h_sc[2], sizeof(DevScalars), hipMemcpyHostToDevice, S.s1),
        "hipMemcpyAsync");
  hipck(hipMemcpyAsync(S.b, b, S.n * 8, hipMemcpyDeviceToDevice, S.s1), "hipMemcpyAsync");
  if (S.block) {          // the iterate of A M^-1 y = b: y_0 = M x_0
    launch_apply_op(S, S.Mb, x, S.x, S.s1);
    hipck(hipGetLastError(), "block-Jacobi y_0 launch");
  } else {
    hipck(hipMemcpyAsync(S.x, x, S.n * 8, hipMemcpyDeviceToDevice, S.s1), "hipMemcpyAsync");
  }
  hipck(hipEventRecord(S.ev_t0, S.s1), "hipEventRecord");
}

void end_solve(Solver& S, double* x, hipStream_t cs) {
  if (S.block) {          // x = M^-1 y
    launch_apply_op(S, S.Bi, S.x, x, S.s1);
    hipck(hipGetLastError(), "block-Jacobi x launch");
  } else {
    hipck(hipMemcpyAsync(x, S.x, S.n * 8, hipMemcpyDeviceToDevice, S.s1), "hipMemcpyAsync");
  }
  hipck(hipEventRecord(S.ev_out, S.s1), "hipEventRecord");
  hipck(hipStreamWaitEvent(cs, S.ev_out, 0), "hipStreamWaitEvent");
}

// synchronous read of the device scalars
DevScalars read_scalars(Solver& S) {
  hipck(hipMemcpyAsync(&S.h_sc[0], S.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, S.s1),
        "hipMemcpyAsync");
  hipck(hipStreamSynchronize(S.s1), "hipStreamSynchronize");
  return S.h_sc[0];
}

double true_residual(Solver& S, bool tr) {
  launch_true_res(S, tr, S.s1);
  launch_final(S, FIN_TRUE, 0, S.s1);
  hipck(hipGetLastError(), "true residual launch");
  return read_scalars(S).tr;
}

// One iteration of Algorithm 2 (index i) on stream st.
//
// Structured operators (fused_kind != 0): phase A computes t_i = A M^-1 w_i
// and phase B v_i = A M^-1 z_i themselves, and phase B runs the GLRED 1
// final in its prologue.  Without the automated criterion the GLRED 2 final
// of an iteration is left to the next phase A's prologue (the return value
// says so; `pending` passes it on), except in the last iteration of a chunk
// and before a gap measurement, which end with the GLRED 2 final as a kernel
// of its own: the scalars the host polls between chunks are then complete.
// Other operators: the two SPMVs are kernels of their own and carry the
// finals in their first blocks, overlapped with the product.
bool enqueue_iteration(Solver& S, bool tr, int i, const pbcg_opts& o, hipStream_t st,
                       bool pending, bool last_of_chunk) {
  const bool fused = fused_kind(S, tr) != 0;
  const bool gap = o.gap_every > 0 && (i + 1) % o.gap_every == 0;
  const bool defer = fused && !o.rr_auto && !last_of_chunk && !gap;
  launch_phaseA(S, tr, pending, st);
  if (!fused) launch_iter_spmv(S, tr, V_Z, V_V, FIN_OMEGA, st);
  launch_phaseB(S, tr, pending, st);
  if (o.rr_auto || (o.rr_period > 0 && (i + 1) % o.rr_period == 0)) {
    launch_rr1(S, tr, false, st);      // predicated on the device (eq:criterion or the period)
    launch_rr2(S, tr, false, st, true, !o.rr_nv);
    if (o.rr_nv) launch_rr3(S, tr, false, st);
  }
  if (!fused) launch_iter_spmv(S, tr, V_W, V_T, FIN_BETA, st);
  else if (!defer) launch_fin(S, FIN_BETA, st);
  launch_bound_products(S, st);
  if (gap) {
    launch_gap(S, tr, st);
    launch_final(S, FIN_GAP, 0, st);
  }
  return defer;
}

// iterations start .. start + len - 1 as one chunk
void enqueue_chunk(Solver& S, bool tr, int start, int len, const pbcg_opts& o, hipStream_t st) {
  bool pending = false;
  for (int j = 0; j < len; ++j)
    pending = enqueue_iteration(S, tr, start + j, o, st, pending, j == len - 1);
}

hipGraphExec_t chunk_graph(Solver& S, bool tr, int start, int len, const pbcg_opts& o) {
  const int off = (o.rr_period > 0 && !o.rr_auto) ? start % o.rr_period : 0;
  const std::string key = std::to_string(tr) + "/" + std::to_string(o.rr_auto) + "/" +
                          std::to_string(len) + "/" +
                          std::to_string(off) + "/" + std::to_string(o.rr_period) + "/" +
                          std::to_string(o.gap_every > 0 ? start % o.gap_every : 0) + "/" +
                          std::to_string(o.gap_every) + "/" + std::to_string(o.rr_nv ? 1 : 0);
  auto it = S.graphs.find(key);
  if (it != S.graphs.end()) return it->second;
  hipGraph_t g = nullptr;
  hipck(hipStreamBeginCapture(S.s1, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  enqueue_chunk(S, tr, start, len, o, S.s1);
  hipck(hipStreamEndCapture(S.s1, &g), "hipStreamEndCapture");
  hipGraphExec_t ge = nullptr;
  hipck(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0), "hipGraphInstantiate");
  hipck(hipGraphDestroy(g), "hipGraphDestroy");
  S.graphs[key] = ge;
  return ge;
}

// Runs iterations until the device reports done or `maxit` iterations have
// been completed.  Returns the device scalars after draining the stream.
DevScalars run_iterations(Solver& S, bool tr, int start, const pbcg_opts& o) {
  // a chunk ends with a host poll (a copy of the scalars and an event) and,
  // with graphs, a graph launch: about 15 us per chunk, so graph chunks are
  // long (the early-exit launches after convergence cost ~1 us each)
  int K = o.check_every > 0 ? o.check_every : (o.use_graph ? 32 : 8);
  // With periodic replacement a chunk is a whole number of periods or a
  // divisor of the period, so that one or a few captured variants serve the
  // whole solve.  By default: as many periods as fit in 128 iterations
  // (1000^2 Poisson, every 50, ms per 1000 iterations: chunks of 25 39.6, 50
  // 39.0, 100 38.8, 200 38.75; a longer chunk costs only the early-exit
  // launches after convergence), for longer periods the longest divisor up to
  // 64; a requested polling interval is kept if it is a multiple of the
  // period, else the closest divisor is taken.  Without periodic replacement
  // chunks stay at 32 (automated strategy, 1000^2 Poisson to 1e-10: 32 and 64
  // 251.7 ms, 128 254.0 ms: after a stop or restart the early-exit launches
  // of up to two chunks cost more than the fewer chunk ends save).
  if (o.use_graph && o.rr_period > 0 && !o.rr_auto) {
    if (o.check_every > 0 && o.check_every % o.rr_period == 0) {
      K = o.check_every;
    } else if (o.check_every <= 0 && o.rr_period <= 128) {
      K = o.rr_period * (128 / o.rr_period);
    } else {
      int best = 1;
      for (int d = 1; d <= std::min(o.rr_period, 64); ++d)
        if (o.rr_period % d == 0 &&
            (o.check_every > 0 ? std::abs(d - K) < std::abs(best - K) : d > best))
          best = d;
      K = best;
    }
  }
  int it = start;
  int chunk = 0;
  bool outstanding = false;
  while (it < o.maxit) {
    const int len = std::min(K, o.maxit - it);
    if (o.use_graph) {
      hipGraphExec_t ge = chunk_graph(S, tr, it, len, o);
      hipck(hipGraphLaunch(ge, S.s1), "hipGraphLaunch");
    } else {
      enqueue_chunk(S, tr, it, len, o, S.s1);
    }
    hipck(hipGetLastError(), "iteration launch");
    it += len;
    const int slot = chunk & 1;
    hipck(hipMemcpyAsync(&S.h_sc[slot], S.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, S.s1),
          "hipMemcpyAsync");
    hipck(hipEventRecord(S.ev_poll[slot], S.s1), "hipEventRecord");
    if (outstanding) {
      const int prev = (chunk - 1) & 1;
      hipck(hipEventSynchronize(S.ev_poll[prev]), "hipEventSynchronize");
      if (S.h_sc[prev].done != RUNNING) break;
    }
    outstanding = true;
    ++chunk;
  }
  return read_scalars(S);
}

int finish_stats(Solver& S, bool tr, const DevScalars& d, int status, pbcg_stats* st,
                 double tr_norm, int spmvs) {
  hipck(hipEventRecord(S.ev_t1, S.s1), "hipEventRecord");
  hipck(hipEventSynchronize(S.ev_t1), "hipEventSynchronize");
  float ms = 0.0f;
  hipck(hipEventElapsedTime(&ms, S.ev_t0, S.ev_t1), "hipEventElapsedTime");
  if (st) {
    st->status = status;
    st->iterations = d.iter;
    st->replacements = d.rr_count;
    st->spmvs = spmvs;
    st->bnorm = d.nb;
    st->rnorm0 = d.rn0;
    st->rel_res_recursive = d.nb > 0 ? d.rn / d.nb : 0.0;
    st->rel_res_true = d.nb > 0 ? tr_norm / d.nb : 0.0;
    st->elapsed_ms = ms;
    st->single_kernel = 0;
  }
  (void)tr;
  return status;
}

// What block-Jacobi handles (which store A M^-1) cannot do.
void check_block(const Solver& S, bool transpose, bool rr_auto) {
  if (!S.block) return;
  if (transpose)
    fail(PBCG_ERR_UNSUPPORTED, "block-Jacobi handles do not solve with the transpose");
  if (rr_auto)
    fail(PBCG_ERR_UNSUPPORTED, "block-Jacobi handles do not support the automated replacement");
}

int solve_pipelined(Solver& S, const double* b, double* x, const pbcg_opts& o, pbcg_stats* st) {
  validate_opts(o);
  check_block(S, o.transpose != 0, o.rr_auto != 0);
  const bool tr = o.transpose != 0;
  S.auto_rr = o.rr_auto != 0;
  S.bound_prod = o.rr_auto >= 3;
  if (tr) build_transpose(S);
  hipStream_t cs = (hipStream_t)o.stream;
  begin_solve(S, b, x, o, cs);
  hipError_t sk_err = hipSuccess;
  if (o.single_kernel && launch_small_solve(S, o, S.s1, &sk_err)) {
    hipck(sk_err, "single-kernel solve: hipFuncSetAttribute");
    hipck(hipGetLastError(), "single-kernel solve launch");
    const double trn = true_residual(S, tr);
    const DevScalars d = read_scalars(S);
    const int spmvs = 3 + 2 * d.iter + (o.rr_nv ? 5 : 4) * d.rr_count + 1;
    end_solve(S, x, cs);
    const int rc = finish_stats(S, tr, d, d.status, st, trn, spmvs);
    if (st) {
      st->restarts = 0;
      st->single_kernel = 1;
    }
    return rc;
  }
  // Algorithm 2 initialisation
  launch_init_res(S, tr, S.s1);
  launch_spmv(S, tr, S.vec[V_R], S.vec[V_W], FIN_NONE, true, S.s1);
  launch_spmv(S, tr, S.vec[V_W], S.vec[V_T], FIN_INIT, false, S.s1);
  launch_bound_products(S, S.s1);
  hipck(hipGetLastError(), "init launch");
  DevScalars d = read_scalars(S);
  int status = -1;
  double trn = 0.0;
  int forced = 0;
  int restarts = 0;
  int start = 0;
  if (d.done == STOPPED) {
    status = d.status;
    if (d.nb == 0.0) launch_fill_zero(S, S.x, S.n, 8, S.s1);
  }
  while (status < 0) {
    d = run_iterations(S, tr, start, o);
    // the gap of a stopping iteration: the device skipped it once `done` was
    // raised in that iteration's GLRED 2 final
    if (o.gap_every > 0 && d.iter > 0 && d.iter % o.gap_every == 0 &&
        d.gap_idx < d.iter / o.gap_every) {
      launch_gap(S, tr, S.s1, true);
      launch_final(S, FIN_GAP, 0, S.s1, true);
      hipck(hipGetLastError(), "gap launch");
      d = read_scalars(S);
    }
    if (d.done == STOPPED && d.status == PBCG_BREAKDOWN_RHO && restarts < o.restarts &&
        d.iter < o.maxit) {
      // start again from the current x (option; not part of the paper's method)
      ++restarts;
      launch_set_done(S, RUNNING, S.s1);
      launch_init_res(S, tr, S.s1);
      launch_spmv(S, tr, S.vec[V_R], S.vec[V_W], FIN_NONE, true, S.s1);
      launch_spmv(S, tr, S.vec[V_W], S.vec[V_T], FIN_INIT, false, S.s1);
      launch_bound_products(S, S.s1);
      hipck(hipGetLastError(), "restart launch");
      d = read_scalars(S);
      if (d.done != STOPPED) {
        start = d.iter;
        continue;
      }
    }
    if (d.done == STOPPED) {
      status = d.status;
      break;
    }
    if (d.done == RUNNING) {  // maxit reached without a device-side stop
      status = PBCG_MAXIT;
      break;
    }
    // recursive residual met the tolerance: confirm on the true residual
    trn = true_residual(S, tr);
    d = read_scalars(S);
    if (trn <= o.tol * d.nb) {
      status = PBCG_CONVERGED;
      break;
    }
    if ((o.rr_period <= 0 && !o.rr_auto) || forced >= kMaxForcedReplacements) {
      status = PBCG_TRUE_RES_NOT_MET;
      break;
    }
    // replace (eq:rr) and recompute GLRED 2, then continue; the replaced
    // residual is not tested against the tolerance in this iteration.  When a
    // replacement already ran in this iteration, its saved pre-replacement z
    // (for n_i) is kept.
    ++forced;
    const bool save_z = d.n_saved == 0;
    launch_set_done(S, RUNNING, S.s1);
    launch_rr1(S, tr, true, S.s1);
    launch_rr2(S, tr, true, S.s1, save_z, !o.rr_nv);
    if (o.rr_nv) launch_rr3(S, tr, true, S.s1);
    launch_spmv(S, tr, S.vec[V_W], S.vec[V_T], FIN_REDO, false, S.s1);
    launch_bound_products(S, S.s1);
    hipck(hipGetLastError(), "replacement launch");
    d = read_scalars(S);
    if (d.done == STOPPED) {
      status = d.status;
      break;
    }
    start = d.iter;
    if (start >= o.maxit) {
      status = PBCG_MAXIT;
      break;
    }
  }
  trn = true_residual(S, tr);
  d = read_scalars(S);
  const int spmvs = 3 * (1 + restarts) + 2 * d.iter + (o.rr_nv ? 5 : 4) * d.rr_count + 1;
  end_solve(S, x, cs);
  const int rc = finish_stats(S, tr, d, status, st, trn, spmvs);
  if (st) st->restarts = restarts;
  return rc;
}

int solve_classic(Solver& S, const double* b, double* x, const pbcg_opts& o, pbcg_stats* st) {
  validate_opts(o);
  check_block(S, o.transpose != 0, false);
  S.auto_rr = false;
  S.bound_prod = false;
  const bool tr = o.transpose != 0;
  if (tr) build_transpose(S);
  hipStream_t cs = (hipStream_t)o.stream;
  begin_solve(S, b, x, o, cs);
  launch_cl_init(S, tr, S.s1);
  launch_final(S, FIN_C_INIT, 0, S.s1);
  hipck(hipGetLastError(), "init launch");
  DevScalars d = read_scalars(S);
  int status = -1;
  if (d.done == STOPPED) {
    status = d.status;
    if (d.nb == 0.0) launch_fill_zero(S, S.x, S.n, 8, S.s1);
  } else {
    const int K = o.check_every > 0 ? o.check_every : 8;
    int it = 0, chunk = 0;
    bool outstanding = false;
    while (it < o.maxit) {
      const int len = std::min(K, o.maxit - it);
      for (int j = 0; j < len; ++j) {
        launch_cl_spmv_s(S, tr, S.s1);
        launch_final(S, FIN_C_ALPHA, 0, S.s1);
        launch_cl_spmv_y(S, tr, S.s1);
        launch_final(S, FIN_C_OMEGA, 0, S.s1);
        launch_cl_update(S, S.s1);
        launch_final(S, FIN_C_BETA, 0, S.s1);
        launch_cl_p(S, S.s1);
      }
      hipck(hipGetLastError(), "iteration launch");
      it += len;
      const int slot = chunk & 1;
      hipck(hipMemcpyAsync(&S.h_sc[slot], S.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, S.s1),
            "hipMemcpyAsync");
      hipck(hipEventRecord(S.ev_poll[slot], S.s1), "hipEventRecord");
      if (outstanding) {
        const int prev = (chunk - 1) & 1;
        hipck(hipEventSynchronize(S.ev_poll[prev]), "hipEventSynchronize");
        if (S.h_sc[prev].done != RUNNING) break;
      }
      outstanding = true;
      ++chunk;
    }
    d = read_scalars(S);
    if (d.done == STOPPED) status = d.status;
    else if (d.done == RUNNING) status = PBCG_MAXIT;
    else {
      const double trn = true_residual(S, tr);
      d = read_scalars(S);
      status = trn <= o.tol * d.nb ? PBCG_CONVERGED : PBCG_TRUE_RES_NOT_MET;
    }
  }
  const double trn = true_residual(S, tr);
  d = read_scalars(S);
  end_solve(S, x, cs);
  const int rc = finish_stats(S, tr, d, status, st, trn, 1 + 2 * d.iter + 1);
  if (st) st->restarts = 0;
  return rc;
}

pbcg_opts defaults() {
  pbcg_opts o;
  std::memset(&o, 0, sizeof(o));
  o.tol = 1e-10;
  o.maxit = 10000;
  return o;
}

Solver& H(pbcg_handle h) {
  if (!h) fail(PBCG_ERR_INVALID_ARG, "null handle");
  return h->S;
}

void destroy_solver(pbcg_solver* p) {
  if (!p) return;
  Solver& S = p->S;
  for (auto& kv : S.graphs) (void)hipGraphExecDestroy(kv.second);
  if (S.s1) (void)hipStreamSynchronize(S.s1);
  if (S.h_sc) (void)hipHostFree(S.h_sc);
  hipEvent_t evs[] = {S.ev_in, S.ev_out, S.ev_t0, S.ev_t1, S.ev_poll[0], S.ev_poll[1]};
  for (hipEvent_t e : evs)
    if (e) (void)hipEventDestroy(e);
  if (S.s1) (void)hipStreamDestroy(S.s1);
  delete p;
}

// ----------------------------------------------------------------------------
// Reduction scratch of pbicgstab_solve_noalloc: the partial sums (kNumSlots x
// kMaxPartials doubles) and the two device scalar structs, in a static device
// array (each GPU the library runs on holds its own copy until the process
// ends).  Host code never passes `scratch` itself to a kernel: its device
// address comes from hipGetSymbolAddress, once per device.
// ----------------------------------------------------------------------------

constexpr size_t kScratchPartialBytes = sizeof(double) * kNumSlots * kMaxPartials;
constexpr size_t kScratchScalarOffset = (kScratchPartialBytes + kWsAlign - 1) / kWsAlign * kWsAlign;
constexpr size_t kScratchBytes =
    kScratchScalarOffset + (2 * sizeof(DevScalars) + kWsAlign - 1) / kWsAlign * kWsAlign;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device.
char* scratch_address() {
  int dev = -1;
  hipck(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) fail(PBCG_ERR_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    hipck(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) fail(PBCG_ERR_HIP, "hipGetSymbolAddress(scratch) returned null");
    g_scratch_addr[dev] = p;
  }
  return (char*)g_scratch_addr[dev];
}

// Points a handle's reduction scratch at the static array for the lifetime
// of the object (restored on every exit path).
struct ScratchSwap {
  Solver& S;
  double* partials;
  DevScalars* sc;
  ScratchSwap(Solver& s, char* base) : S(s), partials(s.partials), sc(s.sc) {
    S.partials = (double*)base;
    S.sc = (DevScalars*)(base + kScratchScalarOffset);
  }
  ~ScratchSwap() {
    S.partials = partials;
    S.sc = sc;
  }
};

}  // namespace

// ----------------------------------------------------------------------------
// C ABI
// ----------------------------------------------------------------------------

extern "C" {

void pbicgstab_default_opts(pbcg_opts* opt) {
  if (opt) *opt = defaults();
}

size_t pbicgstab_workspace_bytes(int format, int64_t n, int64_t nnz, int32_t width,
                                 int precision, int precond, int with_transpose) {
  g_last_error.clear();
  const bool csr = format == PBCG_CSR;
  if ((!csr && format != PBCG_ST_2D5 && format != PBCG_ST_3D7 && format != PBCG_ST_DIA5) ||
      n < 1 || n > (int64_t)2000000000 || (csr && (nnz < 0 || width < 0)) ||
      (precision != PBCG_FP64 && precision != PBCG_MIXED) ||
      (precond != PBCG_PC_NONE && precond != PBCG_PC_JACOBI &&
       !(csr && block_size_of(precond) > 0))) {
    g_last_error = "pbicgstab_workspace_bytes: invalid arguments";
    return 0;
  }
  return layout_bytes(format, n, nnz, width, precision, precond, with_transpose != 0);
}

int pbicgstab_create_csr(pbcg_handle* out, int64_t n, int64_t nnz, const int32_t* rowptr_d,
                         const int32_t* col_d, const double* val_d, int precision, int precond,
                         void* workspace, size_t ws_bytes, void* stream) {
  return guarded([&]() -> int {
    if (!out) fail(PBCG_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (n < 1) fail(PBCG_ERR_INVALID_ARG, "n must be >= 1");
    if (nnz < 0 || nnz > (int64_t)2000000000) fail(PBCG_ERR_INVALID_ARG, "nnz out of range");
    if (!rowptr_d || (nnz > 0 && (!col_d || !val_d))) fail(PBCG_ERR_INVALID_ARG, "null CSR array");
    hipStream_t cs = (hipStream_t)stream;
    hipck(hipStreamSynchronize(cs), "hipStreamSynchronize");
    // the CSR arrays are read once, on the host, where the layout is built
    std::vector<int32_t> rowptr(n + 1), col(nnz);
    std::vector<double> val(nnz);
    hipck(hipMemcpy(rowptr.data(), rowptr_d, (n + 1) * 4, hipMemcpyDeviceToHost), "hipMemcpy");
    if (nnz > 0) {
      hipck(hipMemcpy(col.data(), col_d, nnz * 4, hipMemcpyDeviceToHost), "hipMemcpy");
      hipck(hipMemcpy(val.data(), val_d, nnz * 8, hipMemcpyDeviceToHost), "hipMemcpy");
    }
    if (rowptr[0] != 0 || rowptr[n] != nnz) fail(PBCG_ERR_INVALID_ARG, "rowptr[0] must be 0 and rowptr[n] == nnz");
    for (int64_t i = 0; i < n; ++i)
      if (rowptr[i + 1] < rowptr[i]) fail(PBCG_ERR_INVALID_ARG, "rowptr must be nondecreasing");
    for (int64_t kk = 0; kk < nnz; ++kk)
      if (col[kk] < 0 || col[kk] >= n) fail(PBCG_ERR_INVALID_ARG, "column index out of range");
    const int bs = (int)block_size_of(precond);
    auto* p = new pbcg_solver();
    try {
      Solver& S = p->S;
      S.n = n;
      S.nnz = nnz;
      S.kind = OP_SELL;
      common_setup(S, precision, bs > 0 ? PBCG_PC_NONE : precond, workspace, ws_bytes);
      if (bs > 0) {
        // block-Jacobi: the handle iterates on A M^-1 (see setup_block_jacobi)
        setup_block_jacobi(S, bs, rowptr, col, val);
        S.h_rowptr = std::move(rowptr);
        S.h_col = std::move(col);
        S.h_val = std::move(val);
        norms_csr(S);
        hipck(hipDeviceSynchronize(), "hipDeviceSynchronize");
        *out = p;
        return PBCG_OK;
      }
      S.h_rowptr = std::move(rowptr);
      S.h_col = std::move(col);
      S.h_val = std::move(val);
      std::vector<int64_t> sptr;
      std::vector<int32_t> scol;
      std::vector<double> sval;
      int mw = 0;
      build_sell(n, S.h_rowptr.data(), S.h_col.data(), S.h_val.data(), sptr, scol, sval, S.h_pos,
                 mw);
      upload_sell(S, S.A, sptr, scol, sval, mw);
      S.d_posA = (int64_t*)dalloc(S, std::max<int64_t>(nnz, 1) * 8);
      hipck(hipMemcpy(S.d_posA, S.h_pos.data(), nnz * 8, hipMemcpyHostToDevice), "hipMemcpy");
      S.d_rowptr = (int32_t*)dalloc(S, (n + 1) * 4);
      S.d_col = (int32_t*)dalloc(S, std::max<int64_t>(nnz, 1) * 4);
      hipck(hipMemcpy(S.d_rowptr, S.h_rowptr.data(), (n + 1) * 4, hipMemcpyHostToDevice),
            "hipMemcpy");
      hipck(hipMemcpy(S.d_col, S.h_col.data(), nnz * 4, hipMemcpyHostToDevice), "hipMemcpy");
      set_dinv_csr(S);
      norms_csr(S);
      if (S.dinv) {
        double m = 0.0;
        for (int64_t i = 0; i < n; ++i) {
          double d = 0.0;
          for (int64_t kk = S.h_rowptr[i]; kk < S.h_rowptr[i + 1]; ++kk)
            if (S.h_col[kk] == i) d += S.h_val[kk];
          m = std::max(m, std::fabs(1.0 / d));
        }
        S.normM = m;
      }
      hipck(hipDeviceSynchronize(), "hipDeviceSynchronize");
    } catch (...) {
      destroy_solver(p);
      throw;
    }
    *out = p;
    return PBCG_OK;
  });
}

int pbicgstab_create_stencil(pbcg_handle* out, int kind, const int64_t* dims,
                             const double* coef_in, int precision, int precond, void* workspace,
                             size_t ws_bytes, void* stream) {
  return guarded([&]() -> int {
    if (!out) fail(PBCG_ERR_INVALID_ARG, "out is null");
    *out = nullptr;
    if (!dims || !coef_in) fail(PBCG_ERR_INVALID_ARG, "dims and coef are required");
    const int nd = kind == PBCG_ST_3D7 ? 3 : 2;
    if (kind != PBCG_ST_2D5 && kind != PBCG_ST_3D7 && kind != PBCG_ST_DIA5)
      fail(PBCG_ERR_INVALID_ARG, "unknown stencil kind");
    int64_t n = 1;
    for (int d = 0; d < nd; ++d) {
      if (dims[d] < 1 || dims[d] > 2000000000) fail(PBCG_ERR_INVALID_ARG, "grid dimension out of range");
      n *= dims[d];
    }
    hipStream_t cs = (hipStream_t)stream;
    hipck(hipStreamSynchronize(cs), "hipStreamSynchronize");
    // constant stencils: host coefficients; DIA5: device rows, read once here
    std::vector<double> dia_host;
    const double* coef = coef_in;
    if (kind == PBCG_ST_DIA5) {
      dia_host.resize(5 * n);
      hipck(hipMemcpy(dia_host.data(), coef_in, 5 * n * 8, hipMemcpyDeviceToHost), "hipMemcpy");
      coef = dia_host.data();
    }
    auto* p = new pbcg_solver();
    try {
      Solver& S = p->S;
      S.n = n;
      S.kind = kind == PBCG_ST_2D5 ? OP_ST2D5 : kind == PBCG_ST_3D7 ? OP_ST3D7 : OP_DIA5;
      common_setup(S, precision, precond, workspace, ws_bytes);
      OpData& o = S.A;
      o.kind = S.kind;
      for (int d = 0; d < nd; ++d) o.dims[d] = (int)dims[d];
      const int64_t nx = dims[0], ny = dims[1], nz = nd == 3 ? dims[2] : 1;
      if (S.kind == OP_ST2D5 || S.kind == OP_ST3D7) {
        const int nc = S.kind == OP_ST2D5 ? 5 : 7;
        for (int d = 0; d < nc; ++d) {
          o.c64[d] = coef[d];
          o.c32[d] = (float)coef[d];
        }
        S.nnz = S.kind == OP_ST2D5 ? 5 * n - 2 * ny - 2 * nx
                                   : 7 * n - 2 * ny * nz - 2 * nx * nz - 2 * nx * ny;
        const double c = coef[S.kind == OP_ST2D5 ? 2 : 3];
        if (precond) {
          if (precision == PBCG_FP64) {
            if (c == 0.0) fail(PBCG_ERR_ZERO_DIAG, "zero stencil centre");
            S.dinv_s = 1.0 / c;
          } else {
            if ((float)c == 0.0f) fail(PBCG_ERR_ZERO_DIAG, "zero stencil centre");
            S.dinv_s = (double)(1.0f / (float)c);
          }
          S.pc = PC_SCALAR;
        }
      } else {
        // DIA5 coefficients, one row of n per direction
        S.h_dia.assign(coef, coef + 5 * n);
        std::vector<double> padded(5 * S.npad, 0.0);
        int64_t nnz = 0;
        for (int d = 0; d < 5; ++d)
          for (int64_t i = 0; i < n; ++i) padded[d * S.npad + i] = coef[d * n + i];
        for (int64_t i = 0; i < n; ++i) {
          const int64_t iy = i / nx, ix = i % nx;
          nnz += 1 + (iy > 0) + (ix > 0) + (ix < nx - 1) + (iy < ny - 1);
        }
        S.nnz = nnz;
        o.dia = dalloc(S, 5 * S.npad * S.tsize);
        if (precision == PBCG_FP64) upload_vals<double>(S, o.dia, padded);
        else upload_vals<float>(S, o.dia, padded);
        if (precond) {
          S.pc = PC_VECTOR;
          S.dinv = dalloc(S, S.npad * S.tsize);
          if (precision == PBCG_FP64) {
            std::vector<double> di(S.npad, 0.0);
            for (int64_t i = 0; i < n; ++i) {
              const double c = coef[2 * n + i];
              if (c == 0.0) fail(PBCG_ERR_ZERO_DIAG, "zero diagonal in row " + std::to_string(i));
              di[i] = 1.0 / c;
            }
            hipck(hipMemcpy(S.dinv, di.data(), S.npad * 8, hipMemcpyHostToDevice), "hipMemcpy");
          } else {
            std::vector<float> di(S.npad, 0.0f);
            for (int64_t i = 0; i < n; ++i) {
              const float c = (float)coef[2 * n + i];
              if (c == 0.0f) fail(PBCG_ERR_ZERO_DIAG, "zero diagonal in row " + std::to_string(i));
              di[i] = 1.0f / c;
            }
            hipck(hipMemcpy(S.dinv, di.data(), S.npad * 4, hipMemcpyHostToDevice), "hipMemcpy");
          }
        }
      }
      (void)nz;
      norms_grid(S, S.kind == OP_DIA5 ? coef : nullptr);
      if (precond) {
        if (S.kind == OP_DIA5) {
          double m = 0.0;
          for (int64_t i = 0; i < n; ++i) m = std::max(m, std::fabs(1.0 / coef[2 * n + i]));
          S.normM = m;
        } else {
          S.normM = std::fabs(1.0 / coef[S.kind == OP_ST2D5 ? 2 : 3]);
        }
      }
      hipck(hipDeviceSynchronize(), "hipDeviceSynchronize");
    } catch (...) {
      destroy_solver(p);
      throw;
    }
    *out = p;
    return PBCG_OK;
  });
}

int pbicgstab_solve(pbcg_handle h, const double* b, double* x, const pbcg_opts* opt,
                    pbcg_stats* st) {
  return guarded([&]() -> int {
    Solver& S = H(h);
    const pbcg_opts o = opt ? *opt : defaults();
    return solve_pipelined(S, b, x, o, st);
  });
}

int pbicgstab_solve_noalloc(pbcg_handle h, const double* b, double* x, const pbcg_opts* opt,
                            pbcg_stats* st) {
  return guarded([&]() -> int {
    Solver& S = H(h);
    pbcg_opts o = opt ? *opt : defaults();
    o.use_graph = 0;                       // instantiating a graph allocates
    if (o.transpose && !S.have_AT)
      fail(PBCG_ERR_UNSUPPORTED,
           "pbicgstab_solve_noalloc: the transposed layout is not built yet (a transposed "
           "pbicgstab_solve or pbicgstab_apply builds it)");
    // every kernel writes the partials of at most kMaxPartials blocks per slot:
    // the scratch holds any handle's reductions, whatever its N
    if (S.nblk > kMaxPartials)
      fail(PBCG_ERR_UNSUPPORTED, "pbicgstab_solve_noalloc: more partial blocks (" +
                                     std::to_string(S.nblk) + ") than the scratch holds (" +
                                     std::to_string(kMaxPartials) + ")");
    char* base = scratch_address();
    ScratchSwap swap(S, base);
    // ordered after the caller's stream, then cleared with a kernel (the array
    // keeps the previous call's contents)
    hipStream_t cs = (hipStream_t)o.stream;
    hipck(hipEventRecord(S.ev_in, cs), "hipEventRecord");
    hipck(hipStreamWaitEvent(S.s1, S.ev_in, 0), "hipStreamWaitEvent");
    launch_fill_zero(S, base, (int64_t)(kScratchBytes / sizeof(double)), sizeof(double), S.s1);
    hipck(hipGetLastError(), "scratch clear launch");
    return solve_pipelined(S, b, x, o, st);
  });
}

int classic_bicgstab_solve(pbcg_handle h, const double* b, double* x, const pbcg_opts* opt,
                           pbcg_stats* st) {
  return guarded([&]() -> int {
    Solver& S = H(h);
    pbcg_opts o = opt ? *opt : defaults();
    o.rr_period = 0;
    o.rr_auto = 0;
    o.gap_every = 0;
    o.use_graph = 0;
    return solve_classic(S, b, x, o, st);
  });
}

int pbicgstab_apply(pbcg_handle h, const double* x, double* y, int transpose, void* stream) {
  return guarded([&]() -> int {
    Solver& S = H(h);
    if (!x || !y) fail(PBCG_ERR_INVALID_ARG, "null vector");
    check_block(S, transpose != 0, false);
    if (transpose) build_transpose(S);
    hipStream_t cs = (hipStream_t)stream;
    hipck(hipEventRecord(S.ev_in, cs), "hipEventRecord");
    hipck(hipStreamWaitEvent(S.s1, S.ev_in, 0), "hipStreamWaitEvent");
    if (S.block) {        // A x = (A M^-1) (M x)
      launch_apply_op(S, S.Mb, x, S.ytmp, S.s1);
      launch_apply(S, false, S.ytmp, y, S.s1);
    } else {
      launch_apply(S, transpose != 0, x, y, S.s1);
    }
    hipck(hipGetLastError(), "apply launch");
    hipck(hipEventRecord(S.ev_out, S.s1), "hipEventRecord");
    hipck(hipStreamWaitEvent(cs, S.ev_out, 0), "hipStreamWaitEvent");
    return PBCG_OK;
  });
}

int pbicgstab_grad_values(pbcg_handle h, const double* lambda, const double* x, double* grad,
                          void* stream) {
  return guarded([&]() -> int {
    Solver& S = H(h);
    if (!lambda || !x || !grad) fail(PBCG_ERR_INVALID_ARG, "null vector");
    if (S.block) fail(PBCG_ERR_UNSUPPORTED, "block-Jacobi handles have no value gradient");
    hipStream_t cs = (hipStream_t)stream;
    hipck(hipEventRecord(S.ev_in, cs), "hipEventRecord");
    hipck(hipStreamWaitEvent(S.s1, S.ev_in, 0), "hipStreamWaitEvent");
    launch_grad(S, lambda, x, grad, S.s1);
    if (S.kind == OP_ST2D5 || S.kind == OP_ST3D7) {
      const int nc = S.kind == OP_ST2D5 ? 5 : 7;
      launch_final(S, FIN_SUM, nc, S.s1);
      hipck(hipMemcpyAsync(grad, &S.sc->sums[0], nc * sizeof(double), hipMemcpyDeviceToDevice,
                           S.s1), "hipMemcpyAsync");
    }
    hipck(hipGetLastError(), "grad launch");
    hipck(hipEventRecord(S.ev_out, S.s1), "hipEventRecord");
    hipck(hipStreamWaitEvent(cs, S.ev_out, 0), "hipStreamWaitEvent");
    return PBCG_OK;
  });
}

int pbicgstab_update_values(pbcg_handle h, const double* values, int on_device, void* stream) {
  return guarded([&]() -> int {
    Solver& S = H(h);
    if (!values) fail(PBCG_ERR_INVALID_ARG, "null values");
    if (S.block) fail(PBCG_ERR_UNSUPPORTED, "block-Jacobi handles do not update values");
    hipStream_t cs = (hipStream_t)stream;
    hipck(hipStreamSynchronize(cs), "hipStreamSynchronize");
    hipck(hipStreamSynchronize(S.s1), "hipStreamSynchronize");
    if (S.kind == OP_SELL) {
      if (on_device) {
        // scattered into the layouts on the device (values, Jacobi diagonal, A^T)
        hipck(hipMemsetAsync(&S.sc->bad_diag, 0, sizeof(int32_t), S.s1), "hipMemsetAsync");
        launch_update_sell(S, values, S.s1);
        hipck(hipGetLastError(), "update launch");
        hipck(hipStreamSynchronize(S.s1), "hipStreamSynchronize");
        // the host copy stays current for a later transpose build and the norm bounds
        hipck(hipMemcpy(S.h_val.data(), values, S.nnz * 8, hipMemcpyDeviceToHost), "hipMemcpy");
        int32_t bad = 0;
        hipck(hipMemcpy(&bad, &S.sc->bad_diag, 4, hipMemcpyDeviceToHost), "hipMemcpy");
        if (bad) fail(PBCG_ERR_ZERO_DIAG, "zero diagonal after value update");
      } else {
        // host values: scattered on the host and uploaded (no device staging)
        std::memcpy(S.h_val.data(), values, S.nnz * 8);
        upload_scattered(S, S.A, S.h_pos);
        if (S.have_AT) upload_scattered(S, S.AT, S.h_posAT);
        if (S.precond) upload_dinv_csr(S);
      }
      norms_csr(S);
      return PBCG_OK;
    }
    if (S.kind == OP_ST2D5 || S.kind == OP_ST3D7) {
      const int nc = S.kind == OP_ST2D5 ? 5 : 7;
      double c[7];
      if (on_device) hipck(hipMemcpy(c, values, nc * 8, hipMemcpyDeviceToHost), "hipMemcpy");
      else std::memcpy(c, values, nc * 8);
      const double centre = c[nc / 2];
      if (S.precond && (S.precision == PBCG_FP64 ? centre == 0.0 : (float)centre == 0.0f))
        fail(PBCG_ERR_ZERO_DIAG, "zero stencil centre");
      for (int d = 0; d < nc; ++d) {
        S.A.c64[d] = c[d];
        S.A.c32[d] = (float)c[d];
      }
      if (S.precond) {
        S.dinv_s = S.precision == PBCG_FP64 ? 1.0 / centre : (double)(1.0f / (float)centre);
        S.normM = std::fabs(1.0 / centre);
      }
      norms_grid(S, nullptr);
      if (S.have_AT) {
        S.have_AT = false;
        build_transpose(S);
      }
      for (auto& kv : S.graphs) (void)hipGraphExecDestroy(kv.second);
      S.graphs.clear();
      return PBCG_OK;
    }
    // DIA5
    std::vector<double> host(5 * S.n);
    if (on_device) hipck(hipMemcpy(host.data(), values, 5 * S.n * 8, hipMemcpyDeviceToHost), "hipMemcpy");
    else std::memcpy(host.data(), values, 5 * S.n * 8);
    std::vector<double> padded(5 * S.npad, 0.0);
    for (int d = 0; d < 5; ++d)
      for (int64_t i = 0; i < S.n; ++i) padded[d * S.npad + i] = host[d * S.n + i];
    if (S.precision == PBCG_FP64) upload_vals<double>(S, S.A.dia, padded);
    else upload_vals<float>(S, S.A.dia, padded);
    if (S.precond) {
      std::vector<double> di(S.npad, 0.0);
      for (int64_t i = 0; i < S.n; ++i) {
        const double c = host[2 * S.n + i];
        if (S.precision == PBCG_FP64) {
          if (c == 0.0) fail(PBCG_ERR_ZERO_DIAG, "zero diagonal after value update");
          di[i] = 1.0 / c;
        } else {
          if ((float)c == 0.0f) fail(PBCG_ERR_ZERO_DIAG, "zero diagonal after value update");
          di[i] = (double)(1.0f / (float)c);
        }
      }
      if (S.precision == PBCG_FP64) upload_vals<double>(S, S.dinv, di);
      else upload_vals<float>(S, S.dinv, di);
    }
    S.h_dia = host;
    norms_grid(S, S.h_dia.data());
    if (S.have_AT) {
      launch_dia5_transpose(S, S.s1);
      hipck(hipStreamSynchronize(S.s1), "hipStreamSynchronize");
    }
    return PBCG_OK;
  });
}

int pbicgstab_dia5_assemble_kappa(pbcg_handle h, const double* kappa, double cx, double cy,
                                  double hgrid, void* stream) {
  return guarded([&]() -> int {
    Solver& S = H(h);
    if (S.kind != OP_DIA5) fail(PBCG_ERR_UNSUPPORTED, "not a DIA5 handle");
    if (!kappa) fail(PBCG_ERR_INVALID_ARG, "null kappa");
    if (S.precond && !S.dinv) fail(PBCG_ERR_INVALID_ARG, "no Jacobi diagonal");
    hipStream_t cs = (hipStream_t)stream;
    hipck(hipEventRecord(S.ev_in, cs), "hipEventRecord");
    hipck(hipStreamWaitEvent(S.s1, S.ev_in, 0), "hipStreamWaitEvent");
    hipck(hipMemsetAsync(&S.sc->bad_diag, 0, sizeof(int32_t), S.s1), "hipMemsetAsync");
    void* keep = S.dinv;
    if (!S.precond) S.dinv = S.vec[V_TMP];  // assembled diagonal goes to scratch, unused
    launch_kappa_assemble(S, kappa, cx, cy, hgrid, S.s1);
    S.dinv = keep;
    hipck(hipGetLastError(), "assemble launch");
    int32_t bad = 0;
    hipck(hipMemcpyAsync(&bad, &S.sc->bad_diag, 4, hipMemcpyDeviceToHost, S.s1), "hipMemcpyAsync");
    hipck(hipStreamSynchronize(S.s1), "hipStreamSynchronize");
    if (bad && S.precond) fail(PBCG_ERR_ZERO_DIAG, "zero diagonal after assembly");
    refresh_dia5_bounds(S);
    hipck(hipEventRecord(S.ev_out, S.s1), "hipEventRecord");
    hipck(hipStreamWaitEvent(cs, S.ev_out, 0), "hipStreamWaitEvent");
    return PBCG_OK;
  });
}

int pbicgstab_dia5_kappa_grad(pbcg_handle h, const double* lambda, const double* x,
                              double* grad_kappa, void* stream) {
  return guarded([&]() -> int {
    Solver& S = H(h);
    if (S.kind != OP_DIA5) fail(PBCG_ERR_UNSUPPORTED, "not a DIA5 handle");
    if (!lambda || !x || !grad_kappa) fail(PBCG_ERR_INVALID_ARG, "null vector");
    hipStream_t cs = (hipStream_t)stream;
    hipck(hipEventRecord(S.ev_in, cs), "hipEventRecord");
    hipck(hipStreamWaitEvent(S.s1, S.ev_in, 0), "hipStreamWaitEvent");
    launch_kappa_grad(S, lambda, x, grad_kappa, S.s1);
    hipck(hipGetLastError(), "kappa grad launch");
    hipck(hipEventRecord(S.ev_out, S.s1), "hipEventRecord");
    hipck(hipStreamWaitEvent(cs, S.ev_out, 0), "hipStreamWaitEvent");
    return PBCG_OK;
  });
}

int pbicgstab_get_vector(pbcg_handle h, int which, double* out, void* stream) {
  return guarded([&]() -> int {
    Solver& S = H(h);
    if (!out) fail(PBCG_ERR_INVALID_ARG, "null output");
    if (which < 0 || which > 11) fail(PBCG_ERR_INVALID_ARG, "unknown vector id");
    hipStream_t cs = (hipStream_t)stream;
    hipck(hipEventRecord(S.ev_in, cs), "hipEventRecord");
    hipck(hipStreamWaitEvent(S.s1, S.ev_in, 0), "hipStreamWaitEvent");
    if (which <= 9) {
      launch_to_double(S, S.vec[which], out, S.n, S.s1);
    } else if (which == 10) {
      hipck(hipMemcpyAsync(out, S.x, S.n * 8, hipMemcpyDeviceToDevice, S.s1), "hipMemcpyAsync");
    } else {
      if (S.pc == PC_VECTOR) {
        launch_to_double(S, S.dinv, out, S.n, S.s1);
      } else {
        std::vector<double> v(S.n, S.pc == PC_SCALAR ? S.dinv_s : 1.0);
        hipck(hipMemcpyAsync(out, v.data(), S.n * 8, hipMemcpyHostToDevice, S.s1), "hipMemcpyAsync");
        hipck(hipStreamSynchronize(S.s1), "hipStreamSynchronize");
      }
    }
    hipck(hipGetLastError(), "get_vector launch");
    hipck(hipEventRecord(S.ev_out, S.s1), "hipEventRecord");
    hipck(hipStreamWaitEvent(cs, S.ev_out, 0), "hipStreamWaitEvent");
    return PBCG_OK;
  });
}

int pbicgstab_time_kernel(pbcg_handle h, int kernel, int reps, double* avg_ms, void* stream) {
  return guarded([&]() -> int {
    Solver& S = H(h);
    if (kernel < 0 || kernel > 7 || reps < 1 || !avg_ms) fail(PBCG_ERR_INVALID_ARG, "bad arguments");
    hipStream_t cs = (hipStream_t)stream;
    hipck(hipEventRecord(S.ev_in, cs), "hipEventRecord");
    hipck(hipStreamWaitEvent(S.s1, S.ev_in, 0), "hipStreamWaitEvent");
    // a state in which every kernel does its full work: scalars of a running
    // iteration with a large tolerance-free budget
    pbcg_opts o = defaults();
    o.tol = 0.0;
    o.maxit = 1 << 30;
    S.auto_rr = false;
    S.bound_prod = false;
    S.h_sc[2] = initial_scalars(S, o, false);
    S.h_sc[2].alpha = 0.5;
    S.h_sc[2].beta = 0.5;
    S.h_sc[2].omega = 0.5;
    S.h_sc[2].omega_prev = 0.5;
    S.h_sc[2].rho = 1.0;
    S.h_sc[2].nb = 1.0;
    hipck(hipMemcpyAsync(S.sc, &S.h_sc[2], sizeof(DevScalars), hipMemcpyHostToDevice, S.s1),
          "hipMemcpyAsync");
    const bool fused = fused_kind(S, false) != 0;
    auto one = [&](int kk) {
      switch (kk) {
        case 0: launch_phaseA(S, false, false, S.s1); break;
        case 1:
          if (fused) launch_fin(S, FIN_OMEGA, S.s1);
          else launch_iter_spmv(S, false, V_Z, V_V, FIN_OMEGA, S.s1);
          break;
        case 2: launch_phaseB(S, false, false, S.s1); break;
        case 3:
          if (fused) launch_fin(S, FIN_PROBE, S.s1);
          else launch_iter_spmv(S, false, V_W, V_T, FIN_PROBE, S.s1);
          break;
        case 5: launch_copy(S, S.x, S.b, S.s1); break;
        case 6: launch_iter_spmv(S, false, V_Z, V_V, FIN_NONE, S.s1); break;
        case 7: launch_fin(S, FIN_PROBE, S.s1); break;
      }
    };
    auto launch = [&]() {
      if (kernel == 4) {
        for (int kk = 0; kk < 4; ++kk)
          if (!(fused && kk == 1)) one(kk);      // phase B carries the GLRED 1 final
      } else {
        one(kernel);
      }
    };
    launch();  // warm-up
    hipck(hipEventRecord(S.ev_t0, S.s1), "hipEventRecord");
    for (int r = 0; r < reps; ++r) launch();
    hipck(hipEventRecord(S.ev_t1, S.s1), "hipEventRecord");
    hipck(hipGetLastError(), "timing launch");
    hipck(hipEventSynchronize(S.ev_t1), "hipEventSynchronize");
    float ms = 0.0f;
    hipck(hipEventElapsedTime(&ms, S.ev_t0, S.ev_t1), "hipEventElapsedTime");
    *avg_ms = (double)ms / reps;
    hipck(hipEventRecord(S.ev_out, S.s1), "hipEventRecord");
    hipck(hipStreamWaitEvent(cs, S.ev_out, 0), "hipStreamWaitEvent");
    return PBCG_OK;
  });
}

int pbicgstab_info(pbcg_handle h, int64_t* n, int64_t* nnz, int64_t* device_bytes) {
  return guarded([&]() -> int {
    Solver& S = H(h);
    if (n) *n = S.n;
    if (nnz) *nnz = S.nnz;
    if (device_bytes) *device_bytes = (int64_t)S.ws_used;
    return PBCG_OK;
  });
}

void pbicgstab_destroy(pbcg_handle h) { destroy_solver(h); }

const char* pbicgstab_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
