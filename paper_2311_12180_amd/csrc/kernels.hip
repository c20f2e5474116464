// Hot-path kernels of restarted PDHG for LP on gfx950 (arXiv 2311.12180).
//
// Every product with K~ or K~' is a row gather over one of the two CSR copies
// (no atomics on values, so results are bitwise reproducible run to run).
// Each pass over a matrix is an "op": what is gathered per nonzero, and what
// the row epilogue does with the row sums (the PDHG updates of eq. (pdhg),
// the eq. (kkt) residuals, the restart, the output).  An op runs in one of two
// layouts, chosen per matrix by timing at create:
//   fused  : row blocks -- runs of short rows whose nonzeros (at most kTile)
//            are streamed once, coalesced, into LDS as products and summed per
//            row by a power-of-two group of lanes, or one long row swept by
//            the whole workgroup -- with the epilogue in the same kernel;
//   panels : phase 1 sums the (row, column-panel) segments with workgroup i
//            serving panel i % 8 only (one XCD per panel, so the gathered
//            slice of the vector stays in that XCD's L2), phase 2 adds each
//            row's segment sums in panel order and runs the epilogue.
// No workgroup reads another workgroup's results inside a launch: reductions
// leave one partial per workgroup and a single-workgroup kernel after the
// launch adds them in a fixed order.
//
//   primal op (rows of K~') : x'_j = proj_[l,u](x_j - (eta/omega)(c_j - (K~'y)_j)), dx_j = x'_j - x_j
//   dual op   (rows of K~)  : y'_i = proj(y_i + eta*omega*(q_i - (K~x)_i - 2(K~dx)_i))
//   k_decide                : the Algorithm 2 step-size decision on the reduced norms
//   eval ops, k_eval_decide : averages, eq. (kkt) on current and average iterate,
//                             Section 4.1 termination, Section 3.4 restart decision
//   restart ops             : apply the restart (new z^{n+1,0}, K~x)
#include <math.h>

#include "pdlp_dev.h"

namespace pdlp {

constexpr int kDecideBlock = 1024;   // threads of the single-workgroup reduction kernels

// ---------------------------------------------------------------------------- helpers

template <typename T>
__device__ __forceinline__ T sel(int c, T a0, T a1) { return c ? a1 : a0; }

// Workgroups are dispatched round-robin over the 8 XCDs; with remap on, each
// XCD gets a contiguous range of row blocks.
__device__ __forceinline__ int logical_block(int nb, int remap) {
  const int i = blockIdx.x;
  if (!remap || nb < 16) return i;
  const int q = nb >> 3, r = nb & 7;
  const int x = i & 7, j = i >> 3;
  return x * q + (x < r ? x : r) + j;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Deterministic workgroup sum over NW wavefronts; the result is valid in
// thread 0 only.  `red` holds NV * NW doubles.
template <int NV, int NW = kBlock / 64>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k * NW + w] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = red[k * NW];
      for (int i = 1; i < NW; ++i) s += red[k * NW + i];
      v[k] = s;
    }
  }
  __syncthreads();
}

template <typename VT>
__device__ __forceinline__ const VT* pick(const double* v, const float* vf);
template <>
__device__ __forceinline__ const double* pick<double>(const double* v, const float*) { return v; }
template <>
__device__ __forceinline__ const float* pick<float>(const double*, const float* vf) { return vf; }

constexpr int kPer = kTile / kBlock;   // nonzeros per thread in one tile

// Loads of one tile of nonzeros [base, base + count) (count <= kTile): each
// thread first issues all of its column and value loads, then all of its
// gathers, so a tile costs two memory round trips per thread instead of two
// per nonzero.  f(e, a, g) receives the tile-relative index, the value and the
// NV gathered entries.
template <int NV, typename VT, class G, class F>
__device__ __forceinline__ void tile_products(const int32_t* __restrict__ ci, const VT* __restrict__ v, int base,
                                              int count, G&& gather, F&& f) {
  if (count <= 0) return;
  // Loads are unconditional (past the end they repeat the last entry, an
  // in-bounds index) so the loop body is straight-line code and every load of
  // the tile is in flight at once; only f is predicated.
  int col[kPer];
  double a[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = (int)threadIdx.x + u * kBlock;
    const int ee = e < count ? e : count - 1;
    col[u] = __builtin_nontemporal_load(&ci[base + ee]);
    a[u] = (double)__builtin_nontemporal_load(&v[base + ee]);
  }
  double g[kPer][NV];
#pragma unroll
  for (int u = 0; u < kPer; ++u) gather(col[u], g[u]);
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = (int)threadIdx.x + u * kBlock;
    if (e < count) f(e, a[u], g[u]);
  }
}

// Row block driver over a CSR-like structure (rp, ci, v): runs `epi(row,
// sums)` exactly once for every row of the block.  Short rows: the products
// val * gathered vector(s) are staged in LDS (coalesced matrix stream), then
// each row is summed by L lanes (L = largest power of two <= 64 with
// L * rows <= kBlock) and the group's first lane runs the epilogue.  A long
// row: the workgroup sweeps it tile by tile (thread t takes entries t, t +
// kBlock, ...), reduces, and thread 0 runs the epilogue.
template <int NV, typename VT, class G, class E>
__device__ __forceinline__ void spmv_block(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                           const VT* __restrict__ v, const RowBlock& rb,
                                           double* __restrict__ lds, double* red, G&& gather, E&& epi) {
  const int r0 = rb.r0, r1 = rb.r1;
  const int e0 = rp[r0];
  const int ne = rp[r1] - e0;
  if (ne > kTile) {
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
    for (int base = e0; base < e0 + ne; base += kTile) {
      const int cnt = min(kTile, e0 + ne - base);
      tile_products<NV, VT>(ci, v, base, cnt, gather, [&](int, double a, const double* g) {
#pragma unroll
        for (int k = 0; k < NV; ++k) s[k] += a * g[k];
      });
    }
    block_sum<NV>(s, red);
    if (threadIdx.x == 0) epi(r0, s);
    return;
  }
  tile_products<NV, VT>(ci, v, e0, ne, gather, [&](int e, double a, const double* g) {
#pragma unroll
    for (int k = 0; k < NV; ++k) lds[k * kTile + e] = a * g[k];
  });
  __syncthreads();
  const int nr = r1 - r0;
  int L = 64;
  while (L > 1 && L * nr > kBlock) L >>= 1;
  const int groups = kBlock / L;
  const int grp = threadIdx.x / L, lane = threadIdx.x - grp * L;
  for (int r = grp; r < nr; r += groups) {
    const int b0 = rp[r0 + r] - e0, b1 = rp[r0 + r + 1] - e0;
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
    for (int e = b0 + lane; e < b1; e += L) {
#pragma unroll
      for (int k = 0; k < NV; ++k) s[k] += lds[k * kTile + e];
    }
    for (int off = L >> 1; off > 0; off >>= 1) {
#pragma unroll
      for (int k = 0; k < NV; ++k) s[k] += __shfl_down(s[k], off, L);
    }
    if (lane == 0) epi(r0 + r, s);
  }
}

__device__ __forceinline__ double proj_lambda(double g, double l, double u) {
  const bool lf = isfinite(l), uf = isfinite(u);
  if (lf && uf) return g;
  if (lf) return g > 0.0 ? g : 0.0;
  if (uf) return g < 0.0 ? g : 0.0;
  return 0.0;
}

__device__ __forceinline__ bool attempt_idle(const DevState* st) {
  return st->done | st->need_eval | st->initial;
}
__device__ __forceinline__ bool eval_idle(const DevState* st) { return st->done | !st->need_eval; }

// ---------------------------------------------------------------------------- ops
//
// An op provides: NV (gathered vectors), NACC (reduced quantities per row
// epilogue), idle(st), mat(p) (which CSR copy), part(p) (its partials or
// nullptr), gather(col, g) and epi(row, s, acc).

// Primal step over the rows of K~' (x-space); adds the previously accepted x
// to the running weighted sum.
struct PrimalOp {
  static constexpr int NV = 1, NACC = 1;
  __device__ static bool idle(const DevState* st) { return attempt_idle(st); }
  __device__ static const DevCsr& mat(const Params& p) { return p.KT; }
  __device__ static double* part(const Params& p) { return p.partA; }
  const double* __restrict__ y;
  const double* __restrict__ x;
  double* __restrict__ xn;
  double* __restrict__ dx;
  double* __restrict__ xsum;
  const double* __restrict__ c;
  const double* __restrict__ lo;
  const double* __restrict__ hi;
  double tau, pw;
  int pend;
  __device__ PrimalOp(const Params& p, const DevState* st) {
    const int cur = st->cur;
    tau = st->eta / st->omega;
    pend = st->has_pending;
    pw = st->pending_w;
    y = sel(cur, p.y[0], p.y[1]);
    x = sel(cur, p.x[0], p.x[1]);
    xn = sel(cur, p.x[1], p.x[0]);
    dx = p.dx;
    xsum = p.xsum;
    c = p.c;
    lo = p.l;
    hi = p.u;
  }
  __device__ void gather(int i, double* g) const { g[0] = y[i]; }
  __device__ void epi(int j, const double* s, double* acc) const {
    const double xj = x[j];
    if (pend) xsum[j] += pw * xj;
    double v = xj - tau * (c[j] - s[0]);
    const double lj = lo[j], uj = hi[j];
    if (v < lj) v = lj;
    if (v > uj) v = uj;
    xn[j] = v;
    const double d = v - xj;
    dx[j] = d;
    acc[0] += d * d;
  }
};

// Dual step over the rows of K~ (y-space).  It gathers dx = x' - x, so K~dx,
// and with it the step bound's denominator dy'K~dx, is a direct product
// rather than the difference of two nearly equal products:
// K~(2x' - x) = K~x + 2 K~dx and K~x' = K~x + K~dx.
struct DualOp {
  static constexpr int NV = 1, NACC = 2;
  __device__ static bool idle(const DevState* st) { return attempt_idle(st); }
  __device__ static const DevCsr& mat(const Params& p) { return p.K; }
  __device__ static double* part(const Params& p) { return p.partB; }
  const double* __restrict__ dx;
  const double* __restrict__ y;
  double* __restrict__ yn;
  const double* __restrict__ kx;
  double* __restrict__ kxn;
  double* __restrict__ ysum;
  const double* __restrict__ q;
  const int8_t* __restrict__ ineq;
  double sigma, pw;
  int pend;
  __device__ DualOp(const Params& p, const DevState* st) {
    const int cur = st->cur;
    sigma = st->eta * st->omega;
    pend = st->has_pending;
    pw = st->pending_w;
    dx = p.dx;
    y = sel(cur, p.y[0], p.y[1]);
    yn = sel(cur, p.y[1], p.y[0]);
    kx = sel(cur, p.kx[0], p.kx[1]);
    kxn = sel(cur, p.kx[1], p.kx[0]);
    ysum = p.ysum;
    q = p.q;
    ineq = p.ineq;
  }
  __device__ void gather(int j, double* g) const { g[0] = dx[j]; }
  __device__ void epi(int i, const double* s, double* acc) const {
    const double yi = y[i];
    if (pend) ysum[i] += pw * yi;
    const double kxo = kx[i], kd = s[0];
    double v = yi + sigma * (q[i] - (kxo + 2.0 * kd));
    if (ineq[i] && v < 0.0) v = 0.0;
    yn[i] = v;
    kxn[i] = kxo + kd;
    const double d = v - yi;
    acc[0] += d * d;
    acc[1] += d * kd;
  }
};

// Rows of K~ in an evaluation: K~x and K~x_bar (FP64 matrix), the primal
// residual of eq. (kkt) (scaled, and unscaled by D1^-1 for Section 4.1), q'y,
// q'y_bar, ||y - y0||^2, ||y_bar - y0||^2; forms y_bar (flushing the pending weight).
struct EvalRowsOp {
  static constexpr int NV = 2, NACC = 8;
  __device__ static bool idle(const DevState* st) { return eval_idle(st); }
  __device__ static const DevCsr& mat(const Params& p) { return p.K; }
  __device__ static double* part(const Params& p) { return p.partE1; }
  const Params* pp;
  const double* __restrict__ x;
  const double* __restrict__ xb;
  const double* __restrict__ y;
  double pw, se;
  int init, pend;
  __device__ EvalRowsOp(const Params& p, const DevState* st) : pp(&p) {
    const int cur = st->cur;
    init = st->initial;
    pend = st->has_pending;
    pw = st->pending_w;
    se = st->sum_eta;
    x = sel(cur, p.x[0], p.x[1]);
    xb = p.xbar;
    y = sel(cur, p.y[0], p.y[1]);
  }
  __device__ void gather(int j, double* g) const {
    g[0] = x[j];
    g[1] = xb[j];
  }
  __device__ void epi(int i, const double* s, double* acc) const {
    const Params& p = *pp;
    const double yi = y[i];
    double yb = yi;
    if (!init && se > 0.0) {
      double t = p.ysum[i];
      if (pend) {
        t += pw * yi;
        p.ysum[i] = t;
      }
      yb = t / se;
    }
    p.ybar[i] = yb;
    const double qi = p.q[i], d1 = p.D1[i], y0i = p.y0[i];
    const bool ie = p.ineq[i] != 0;
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const double kv = s[it];
      const double yv = it ? yb : yi;
      double r = kv - qi;
      if (ie) r = (qi - kv) > 0.0 ? (qi - kv) : 0.0;
      acc[0 + it] += r * r;
      const double ru = r / d1;
      acc[2 + it] += ru * ru;
      acc[4 + it] += qi * yv;
      const double dd = yv - y0i;
      acc[6 + it] += dd * dd;
    }
  }
};

// Rows of K~' in an evaluation: K~'y and K~'y_bar (FP64 matrix), lambda =
// proj_Lambda(c - K~'y), the dual residual (scaled, and unscaled by D2^-1),
// l'lambda+ - u'lambda-.
struct EvalColsOp {
  static constexpr int NV = 2, NACC = 6;
  __device__ static bool idle(const DevState* st) { return eval_idle(st); }
  __device__ static const DevCsr& mat(const Params& p) { return p.KT; }
  __device__ static double* part(const Params& p) { return p.partE2; }
  const Params* pp;
  const double* __restrict__ y;
  const double* __restrict__ yb;
  __device__ EvalColsOp(const Params& p, const DevState* st) : pp(&p) {
    const int cur = st->cur;
    y = sel(cur, p.y[0], p.y[1]);
    yb = p.ybar;
  }
  __device__ void gather(int i, double* g) const {
    g[0] = y[i];
    g[1] = yb[i];
  }
  __device__ void epi(int j, const double* s, double* acc) const {
    const Params& p = *pp;
    const double cj = p.c[j], lj = p.l[j], uj = p.u[j], d2 = p.D2[j];
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const double g = cj - s[it];
      const double lam = proj_lambda(g, lj, uj);
      const double rd = g - lam;
      acc[0 + it] += rd * rd;
      const double ru = rd / d2;
      acc[2 + it] += ru * ru;
      const double lp = lam > 0.0 ? lam : 0.0, lm = lam < 0.0 ? -lam : 0.0;
      acc[4 + it] += (lp > 0.0 ? lj * lp : 0.0) - (lm > 0.0 ? uj * lm : 0.0);
    }
  }
};

// y-space part of a restart plus K~x of the new x (in the precision of the
// steps).  The x-space part (k_restart_x) has run before.
struct RestartYOp {
  static constexpr int NV = 1, NACC = 0;
  __device__ static bool idle(const DevState* st) { return !st->restart_flag; }
  __device__ static const DevCsr& mat(const Params& p) { return p.K; }
  __device__ static double* part(const Params&) { return nullptr; }
  const Params* pp;
  const double* __restrict__ x;
  double* __restrict__ y;
  double* __restrict__ kx;
  int cand;
  __device__ RestartYOp(const Params& p, const DevState* st) : pp(&p) {
    const int cur = st->cur;
    cand = st->cand_avg;
    x = sel(cur, p.x[0], p.x[1]);
    y = sel(cur, p.y[0], p.y[1]);
    kx = sel(cur, p.kx[0], p.kx[1]);
  }
  __device__ void gather(int j, double* g) const { g[0] = x[j]; }
  __device__ void epi(int i, const double* s, double*) const {
    const Params& p = *pp;
    const double yc = cand ? p.ybar[i] : y[i];
    y[i] = yc;
    p.y0[i] = yc;
    p.ysum[i] = 0.0;
    kx[i] = s[0];
  }
};

// Output over the rows of K~': x = D2 x~, lambda = D2^-1 proj_Lambda(c~ - K~'y~).
struct OutputOp {
  static constexpr int NV = 1, NACC = 0;
  __device__ static bool idle(const DevState*) { return false; }
  __device__ static const DevCsr& mat(const Params& p) { return p.KT; }
  __device__ static double* part(const Params&) { return nullptr; }
  const Params* pp;
  const double* __restrict__ x;
  const double* __restrict__ y;
  __device__ OutputOp(const Params& p, const DevState* st) : pp(&p) {
    const int cur = st->cur, ra = st->ret_avg;
    x = ra ? p.xbar : sel(cur, p.x[0], p.x[1]);
    y = ra ? p.ybar : sel(cur, p.y[0], p.y[1]);
  }
  __device__ void gather(int i, double* g) const { g[0] = y[i]; }
  __device__ void epi(int j, const double* s, double*) const {
    const Params& p = *pp;
    const double d2 = p.D2[j];
    p.xo[j] = d2 * x[j];
    p.rco[j] = proj_lambda(p.c[j] - s[0], p.l[j], p.u[j]) / d2;
  }
};

// Plain products for the layout tuner: out = K~ in (ProbeK) or K~' in (ProbeKT).
template <int WHICH>
struct ProbeOp {
  static constexpr int NV = 1, NACC = 0;
  __device__ static bool idle(const DevState*) { return false; }
  __device__ static const DevCsr& mat(const Params& p) { return WHICH ? p.KT : p.K; }
  __device__ static double* part(const Params&) { return nullptr; }
  const double* __restrict__ in;
  double* __restrict__ out;
  __device__ ProbeOp(const Params& p, const DevState*) : in(p.probe_in), out(p.probe_out) {}
  __device__ void gather(int j, double* g) const { g[0] = in[j]; }
  __device__ void epi(int i, const double* s, double*) const { out[i] = s[0]; }
};

// ---------------------------------------------------------------------------- generic passes

template <class Op>
struct AccSize {
  static constexpr int N = Op::NACC > 0 ? Op::NACC : 1;
  static constexpr int RED = (Op::NACC > Op::NV ? Op::NACC : Op::NV) * (kBlock / 64);
};

// Fused layout: row blocks, epilogue in the same kernel.
template <class Op, typename VT>
__global__ __launch_bounds__(kBlock) void k_fused(Params p) {
  __shared__ double lds[Op::NV * kTile];
  __shared__ double red[AccSize<Op>::RED];
  if (Op::idle(p.st)) return;
  const Op op(p, p.st);
  const DevCsr& M = Op::mat(p);
  const int b = logical_block(M.nblocks, M.remap);
  double acc[AccSize<Op>::N];
#pragma unroll
  for (int k = 0; k < AccSize<Op>::N; ++k) acc[k] = 0.0;
  spmv_block<Op::NV, VT>(
      M.rp, M.ci, pick<VT>(M.v, M.vf), M.blocks[b], lds, red, [&](int c, double* g) { op.gather(c, g); },
      [&](int r, const double* s) { op.epi(r, s, acc); });
  if constexpr (Op::NACC > 0) {
    block_sum<Op::NACC>(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < Op::NACC; ++k) Op::part(p)[Op::NACC * b + k] = acc[k];
    }
  }
}

// Panel layout, phase 1: segment sums of the blocks of panel blockIdx % 8.
template <class Op, typename VT>
__global__ __launch_bounds__(kBlock) void k_seg(Params p) {
  __shared__ double lds[Op::NV * kTile];
  __shared__ double red[Op::NV * (kBlock / 64)];
  if (Op::idle(p.st)) return;
  const Op op(p, p.st);
  const PanelCsr& S = Op::mat(p).pan;
  double* __restrict__ part = S.part;
  const int32_t* __restrict__ dst = S.seg_dst;
  spmv_block<Op::NV, VT>(
      S.seg_ptr, S.pci, pick<VT>(S.pv, S.pvf), S.sblocks[blockIdx.x], lds, red,
      [&](int c, double* g) { op.gather(c, g); },
      [&](int s, const double* sums) {
        const int d = dst[s];
#pragma unroll
        for (int k = 0; k < Op::NV; ++k) part[Op::NV * d + k] = sums[k];
      });
}

// Panel layout, phase 2: each row adds its segment sums in panel order and
// runs the epilogue; one reduction partial per workgroup of a fixed grid.
template <class Op>
__global__ __launch_bounds__(kBlock) void k_rows(Params p) {
  __shared__ double red[AccSize<Op>::RED];
  if (Op::idle(p.st)) return;
  const Op op(p, p.st);
  const DevCsr& M = Op::mat(p);
  const PanelCsr& S = M.pan;
  double acc[AccSize<Op>::N];
#pragma unroll
  for (int k = 0; k < AccSize<Op>::N; ++k) acc[k] = 0.0;
  for (int r = blockIdx.x * kBlock + threadIdx.x; r < M.nrows; r += gridDim.x * kBlock) {
    double s[Op::NV];
#pragma unroll
    for (int k = 0; k < Op::NV; ++k) s[k] = 0.0;
    for (int q = S.row_seg[r]; q < S.row_seg[r + 1]; ++q) {
#pragma unroll
      for (int k = 0; k < Op::NV; ++k) s[k] += S.part[Op::NV * q + k];
    }
    op.epi(r, s, acc);
  }
  if constexpr (Op::NACC > 0) {
    block_sum<Op::NACC>(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < Op::NACC; ++k) Op::part(p)[Op::NACC * blockIdx.x + k] = acc[k];
    }
  }
}

// ---------------------------------------------------------------------------- decisions

// Algorithm 2 decision on the reduced norms (one thread): eta_bar =
// (omega ||dx||^2 + ||dy||^2 / omega) / (2 |dy'K dx|), eta' = min((1 - (k+2)^-0.3)
// eta_bar, (1 + (k+2)^-0.6) eta); accept when eta <= eta_bar.
__device__ void step_decision(DevState* st, const Params& p, const Trace& tr, double nx, double ny, double dyk) {
  const double eta = st->eta, omega = st->omega;
  const double num = omega * nx + ny / omega;
  const double den = 2.0 * fabs(dyk);
  const double eta_bar = den > 0.0 ? num / den : INFINITY;
  const double kk = (double)(st->k + 2);
  const double a = (1.0 - pow(kk, -0.3)) * eta_bar;
  const double bb = (1.0 + pow(kk, -0.6)) * eta;
  const double eta_next = a < bb ? a : bb;
  const int acc = eta <= eta_bar;
  if (st->n_att < tr.cap) {
    const int64_t s = st->n_att++;
    tr.att_k[s] = st->k;
    tr.att_eta[s] = eta;
    tr.att_etabar[s] = eta_bar;
    tr.att_acc[s] = (int8_t)acc;
  }
  st->attempts++;
  if (!isfinite(num) || isnan(den) || isnan(eta_next)) {
    st->status = 4;
    st->ret_avg = 0;
    st->done = 1;
    return;
  }
  if (acc) {
    st->cur ^= 1;
    st->k++;
    st->t++;
    st->sum_eta += eta;
    st->pending_w = eta;
    st->has_pending = 1;
    st->eta_hat = eta_next;
    st->eta = eta_next;
    if (st->k - st->k_last_eval >= p.P || st->k >= st->max_iter) st->need_eval = 1;
  } else {
    st->has_pending = 0;
    st->eta = eta_next;
  }
}

// Single-workgroup reduction of the step partials and the decision.  It also
// clears the restart flag of the previous evaluation (its restart kernels have run).
__global__ __launch_bounds__(kDecideBlock) void k_decide(Params p) {
  __shared__ double red[3 * (kDecideBlock / 64)];
  DevState* st = p.st;
  if (threadIdx.x == 0 && st->restart_flag) st->restart_flag = 0;
  if (attempt_idle(st)) return;
  double r[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < p.KT.nred; i += kDecideBlock) r[0] += p.partA[i];
  for (int i = threadIdx.x; i < p.K.nred; i += kDecideBlock) {
    r[1] += p.partB[2 * i];
    r[2] += p.partB[2 * i + 1];
  }
  block_sum<3, kDecideBlock / 64>(r, red);
  if (threadIdx.x == 0) step_decision(st, p, p.tr, r[0], r[1], r[2]);
}

// x-space part of the evaluation: flush the pending weight into the sum,
// form x_bar = sum / sum_eta, and reduce c'x, c'x_bar, ||x - x0||^2, ||x_bar - x0||^2.
__global__ __launch_bounds__(kBlock) void k_eval_x(Params p) {
  __shared__ double red[4 * 4];
  const DevState* st = p.st;
  if (eval_idle(st)) return;
  const int cur = st->cur, init = st->initial, pend = st->has_pending;
  const double pw = st->pending_w, se = st->sum_eta;
  const double* __restrict__ x = sel(cur, p.x[0], p.x[1]);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < p.n; j += gridDim.x * kBlock) {
    const double xj = x[j];
    double xb = xj;
    if (!init && se > 0.0) {
      double s = p.xsum[j];
      if (pend) {
        s += pw * xj;
        p.xsum[j] = s;
      }
      xb = s / se;
    }
    p.xbar[j] = xb;
    const double cj = p.c[j], x0j = p.x0[j];
    acc[0] += cj * xj;
    acc[1] += cj * xb;
    double d = xj - x0j;
    acc[2] += d * d;
    d = xb - x0j;
    acc[3] += d * d;
  }
  block_sum<4>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) p.partE0[4 * blockIdx.x + k] = acc[k];
  }
}

// Evaluation decision on the reduced sums S (one thread): termination
// (Section 4.1) on both iterates, else the restart candidate and the restart
// criteria (Section 3.4), the primal weight update (Section 2.2).
__device__ void eval_decision(DevState* st, const Params& p, const Trace& tr, const double* S, double qnorm0,
                              double cnorm0) {
  // S: 0 c'x 1 c'xb 2 |x-x0|^2 3 |xb-x0|^2 | 4,5 rp2 scaled 6,7 rp2 unscaled 8,9 q'y 10,11 |y-y0|^2
  //    | 12,13 rd2 scaled 14,15 rd2 unscaled 16,17 l'lam+ - u'lam-     (pairs: current, average)
  const double omega = st->omega;
  double pobj[2], dobj[2], rel[2], rg[2], rpr[2], rdr[2];
  for (int it = 0; it < 2; ++it) {
    pobj[it] = S[0 + it];
    dobj[it] = S[8 + it] + S[16 + it];
    rg[it] = fabs(dobj[it] - pobj[it]) / (1.0 + fabs(dobj[it]) + fabs(pobj[it]));
    rpr[it] = sqrt(S[6 + it]) / (1.0 + qnorm0);
    rdr[it] = sqrt(S[14 + it]) / (1.0 + cnorm0);
    double r = rg[it];
    if (rpr[it] > r) r = rpr[it];
    if (rdr[it] > r) r = rdr[it];
    if (isnan(rg[it]) || isnan(rpr[it]) || isnan(rdr[it])) r = NAN;
    rel[it] = r;
  }
  auto kkt_w = [&](int it, double om) {
    const double w = p.omega_power == 1 ? om : om * om;
    const double gap = dobj[it] - pobj[it];
    return sqrt(w * S[4 + it] + S[12 + it] / w + gap * gap);
  };
  auto store = [&](int it) {
    st->rel_kkt = rel[it];
    st->rel_gap = rg[it];
    st->rel_p = rpr[it];
    st->rel_d = rdr[it];
    st->pobj = pobj[it];
    st->dobj = dobj[it];
  };
  st->need_eval = 0;
  st->has_pending = 0;
  if (st->initial) {
    st->initial = 0;
    st->kkt0 = kkt_w(0, omega);
    st->kkt_prev = st->kkt0;
    store(0);
    st->ret_avg = 0;
    if (!isfinite(rel[0])) { st->status = 4; st->done = 1; }
    else if (rel[0] <= st->eps_rel) { st->status = 1; st->done = 1; }
    else if (st->max_iter <= 0) { st->status = 2; st->done = 1; }
    st->restart_flag = 1;   // sets z^{0,0} = z, clears the sums, computes K~x
    st->cand_avg = 0;
    return;
  }
  st->evals++;
  st->k_last_eval = st->k;
  const int avg_better = rel[1] < rel[0];
  if (!isfinite(rel[0]) || !isfinite(rel[1])) {
    st->status = 4; st->ret_avg = 0; store(0); st->done = 1;
    return;
  }
  if (rel[0] <= st->eps_rel || rel[1] <= st->eps_rel) {
    st->status = 1; st->ret_avg = avg_better; store(avg_better); st->done = 1;
    return;
  }
  if (st->k >= st->max_iter) {
    st->status = 2; st->ret_avg = avg_better; store(avg_better); st->done = 1;
    return;
  }
  store(avg_better);
  const double kc_cur = kkt_w(0, omega), kc_avg = kkt_w(1, omega);
  // the current iterate only when clearly better: differences at rounding level
  // (e.g. one step into an epoch, where the average is the iterate) go to the average
  const int cand = !(kc_cur < kc_avg - p.tie_rel * kc_avg);
  const double kc = cand ? kc_avg : kc_cur;
  int reason = 0;
  if (kc <= p.beta_suff * st->kkt0) reason = 1;
  else if (kc <= p.beta_nec * st->kkt0 && kc > st->kkt_prev) reason = 2;
  else if ((double)st->t >= p.beta_art * (double)st->k) reason = 3;
  double om = omega;
  if (reason) {
    const double dxn = sqrt(S[2 + cand]), dyn = sqrt(S[10 + cand]);
    if (dxn > p.eps_zero && dyn > p.eps_zero) om = exp(p.theta * log(dyn / dxn) + (1.0 - p.theta) * log(omega));
    st->omega = om;
    st->restart_flag = 1;
    st->cand_avg = cand;
    st->restarts++;
    st->t = 0;
    st->sum_eta = 0.0;
    st->kkt0 = kkt_w(cand, om);
    st->kkt_prev = st->kkt0;
  } else {
    st->kkt_prev = kc;
  }
  if (st->n_eval < tr.cap) {
    const int64_t s = st->n_eval++;
    tr.ev_k[s] = st->k;
    tr.ev_kkt_cur[s] = kc_cur;
    tr.ev_kkt_avg[s] = kc_avg;
    tr.ev_cand[s] = (int8_t)cand;
    tr.ev_reason[s] = (int8_t)reason;
    tr.ev_omega[s] = om;
  }
}

// Single-workgroup reduction of every evaluation partial in a fixed order,
// then the evaluation decision.
__global__ __launch_bounds__(kDecideBlock) void k_eval_decide(Params p, int n_e0_blocks) {
  __shared__ double red[18 * (kDecideBlock / 64)];
  DevState* st = p.st;
  if (eval_idle(st)) return;
  double S[18];
#pragma unroll
  for (int k = 0; k < 18; ++k) S[k] = 0.0;
  for (int i = threadIdx.x; i < n_e0_blocks; i += kDecideBlock) {
#pragma unroll
    for (int k = 0; k < 4; ++k) S[k] += p.partE0[4 * i + k];
  }
  for (int i = threadIdx.x; i < p.K.nred; i += kDecideBlock) {
#pragma unroll
    for (int k = 0; k < 8; ++k) S[4 + k] += p.partE1[8 * i + k];
  }
  for (int i = threadIdx.x; i < p.KT.nred; i += kDecideBlock) {
#pragma unroll
    for (int k = 0; k < 6; ++k) S[12 + k] += p.partE2[6 * i + k];
  }
  block_sum<18, kDecideBlock / 64>(S, red);
  if (threadIdx.x == 0) eval_decision(st, p, p.tr, S, p.qnorm0, p.cnorm0);
}

// x-space part of a restart: z^{n+1,0} = candidate, sums cleared.  The flag
// is cleared by the next k_decide.
__global__ __launch_bounds__(kBlock) void k_restart_x(Params p) {
  const DevState* st = p.st;
  if (!st->restart_flag) return;
  const int cur = st->cur, cand = st->cand_avg;
  double* __restrict__ x = sel(cur, p.x[0], p.x[1]);
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < p.n; j += gridDim.x * kBlock) {
    const double xc = cand ? p.xbar[j] : x[j];
    x[j] = xc;
    p.x0[j] = xc;
    p.xsum[j] = 0.0;
  }
}

// ---------------------------------------------------------------------------- start, output

// Starting point: proj_X(x_start), proj_Y(y_start) in the scaled space; the
// user start (if any) is unscaled: x~ = x / D2, y~ = (LE ? -y : y) / D1.
__global__ __launch_bounds__(kBlock) void k_init_x(Params p, const double* __restrict__ xs) {
  for (int j = blockIdx.x * kBlock + threadIdx.x; j < p.n; j += gridDim.x * kBlock) {
    double v = xs ? xs[j] / p.D2[j] : 0.0;
    if (v < p.l[j]) v = p.l[j];
    if (v > p.u[j]) v = p.u[j];
    p.x[0][j] = v;
    p.x[1][j] = v;
    p.xsum[j] = 0.0;
    p.xbar[j] = v;
    p.x0[j] = v;
    p.dx[j] = 0.0;
  }
}

__global__ __launch_bounds__(kBlock) void k_init_y(Params p, const double* __restrict__ ys) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < p.m; i += gridDim.x * kBlock) {
    double v = 0.0;
    if (ys) {
      v = (p.le[i] ? -ys[i] : ys[i]) / p.D1[i];
      if (p.ineq[i] && v < 0.0) v = 0.0;
    }
    p.y[0][i] = v;
    p.y[1][i] = v;
    p.ysum[i] = 0.0;
    p.ybar[i] = v;
    p.y0[i] = v;
    p.kx[0][i] = 0.0;
    p.kx[1][i] = 0.0;
  }
}

// Output of y = D1 y~, negated back on LE rows.
__global__ __launch_bounds__(kBlock) void k_output_y(Params p) {
  const DevState* st = p.st;
  const int cur = st->cur, ra = st->ret_avg;
  const double* __restrict__ y = ra ? p.ybar : sel(cur, p.y[0], p.y[1]);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < p.m; i += gridDim.x * kBlock) {
    const double v = p.D1[i] * y[i];
    p.yo[i] = p.le[i] ? -v : v;
  }
}

__global__ void k_set_limit(DevState* st, int status) {
  if (!st->done) {
    st->status = status;
    st->ret_avg = 0;
    st->done = 1;
  }
}

// ---------------------------------------------------------------------------- batched LPs
//
// Many independent LPs (packed block-diagonally: LP b owns rows
// [row_off[b], row_off[b+1]) of K~ and columns [col_off[b], col_off[b+1]))
// are solved by one persistent launch.  A workgroup takes the next LP from an
// atomic queue (largest first), runs the whole of Algorithm 1 on it with every
// phase of the single-LP path -- the same ops and the same decision functions
// -- separated by workgroup barriers, keeps the LP's state in LDS, writes the
// solution and takes the next LP.  Rows are swept by groups of L lanes (L per
// LP from the batch schedule: lanes for the rows of K~ and for those of K~').

// Row sweep of one LP's rows [rb, re) with L lanes per row; op.epi runs on the
// group's first lane.
template <int NV, typename VT, class Op>
__device__ __forceinline__ void lane_rows(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                          const VT* __restrict__ v, int rb, int re, int L, const Op& op,
                                          double* acc) {
  const int groups = kBlock / L;
  const int grp = threadIdx.x / L, lane = threadIdx.x - grp * L;
  for (int r = rb + grp; r < re; r += groups) {
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
    const int e1 = rp[r + 1];
    for (int e = rp[r] + lane; e < e1; e += L) {
      const double a = (double)v[e];
      double g[NV];
      op.gather(ci[e], g);
#pragma unroll
      for (int k = 0; k < NV; ++k) s[k] += a * g[k];
    }
    for (int off = L >> 1; off > 0; off >>= 1) {
#pragma unroll
      for (int k = 0; k < NV; ++k) s[k] += __shfl_down(s[k], off, L);
    }
    if (lane == 0) op.epi(r, s, acc);
  }
}

// One pass of an op over an LP's rows: the LDS-tiled row blocks [b0, b1)
// when L = 0 (the single-LP sweep), else rows [rb, re) walked with L lanes per row.
template <int NV, typename VT, class Op>
__device__ __forceinline__ void sweep(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                      const VT* __restrict__ v, const RowBlock* __restrict__ blocks, int b0, int b1,
                                      int rb, int re, int L, const Op& op, double* acc, double* lds, double* red) {
  if (L == 0) {
    for (int j = b0; j < b1; ++j) {
      spmv_block<NV, VT>(rp, ci, v, blocks[j], lds, red, [&](int c, double* g) { op.gather(c, g); },
                         [&](int r, const double* s) { op.epi(r, s, acc); });
      __syncthreads();
    }
  } else {
    lane_rows<NV, VT>(rp, ci, v, rb, re, L, op, acc);
  }
}

__device__ void batch_solve_one(const Params& p, const BatchParams& bp, int b, DevState* S, double* red,
                                double* lds) {
  const int r0 = bp.row_off[b], r1 = bp.row_off[b + 1];
  const int c0 = bp.col_off[b], c1 = bp.col_off[b + 1];
  const int LK = bp.lanes[2 * b], LT = bp.lanes[2 * b + 1];
  const int k0 = bp.bk_off[b], k1 = bp.bk_off[b + 1], t0 = bp.bt_off[b], t1 = bp.bt_off[b + 1];
  const Trace tr = b == bp.trace_lp ? p.tr : Trace{};
  const double qn0 = sqrt(bp.norms[4 * b]), cn0 = sqrt(bp.norms[4 * b + 1]);
  const bool f32 = p.use_f32 != 0;
  if (threadIdx.x == 0) {
    DevState z{};
    *S = z;
    const double km = bp.kmax[b];
    S->eta = S->eta_hat = km > 0.0 ? 1.0 / km : 1.0;
    const double cn = sqrt(bp.norms[4 * b + 2]), qn = sqrt(bp.norms[4 * b + 3]);
    const double w0 = (cn > bp.eps_zero && qn > bp.eps_zero) ? cn / qn : 1.0;
    S->omega = bp.omega_warm[b] > 0.0 ? bp.omega_warm[b] : w0;
    S->initial = 1;
    S->need_eval = 1;
    S->eps_rel = bp.eps_rel;
    S->max_iter = bp.max_iter;
  }
  // starting point (as k_init_x / k_init_y)
  const bool warm = bp.warm[b] != 0;
  for (int j = c0 + threadIdx.x; j < c1; j += kBlock) {
    double v = warm ? bp.wx[j] / p.D2[j] : 0.0;
    if (v < p.l[j]) v = p.l[j];
    if (v > p.u[j]) v = p.u[j];
    p.x[0][j] = v;
    p.x[1][j] = v;
    p.xsum[j] = 0.0;
    p.xbar[j] = v;
    p.x0[j] = v;
    p.dx[j] = 0.0;
  }
  for (int i = r0 + threadIdx.x; i < r1; i += kBlock) {
    double v = 0.0;
    if (warm) {
      v = (p.le[i] ? -bp.wy[i] : bp.wy[i]) / p.D1[i];
      if (p.ineq[i] && v < 0.0) v = 0.0;
    }
    p.y[0][i] = v;
    p.y[1][i] = v;
    p.ysum[i] = 0.0;
    p.ybar[i] = v;
    p.y0[i] = v;
    p.kx[0][i] = 0.0;
    p.kx[1][i] = 0.0;
  }
  __syncthreads();
  int64_t k_seen = 0, rejected = 0;  // thread 0: accepted steps at the last attempt, rejections since
  for (;;) {
    if (S->need_eval) {
      // --- evaluation: averages, eq. (kkt) pieces, Section 4.1 quantities
      double acc[18];
#pragma unroll
      for (int k = 0; k < 18; ++k) acc[k] = 0.0;
      {
        const int cur = S->cur, init = S->initial, pend = S->has_pending;
        const double pw = S->pending_w, se = S->sum_eta;
        const double* __restrict__ x = sel(cur, p.x[0], p.x[1]);
        for (int j = c0 + threadIdx.x; j < c1; j += kBlock) {
          const double xj = x[j];
          double xb = xj;
          if (!init && se > 0.0) {
            double s = p.xsum[j];
            if (pend) {
              s += pw * xj;
              p.xsum[j] = s;
            }
            xb = s / se;
          }
          p.xbar[j] = xb;
          const double cj = p.c[j], x0j = p.x0[j];
          acc[0] += cj * xj;
          acc[1] += cj * xb;
          double d = xj - x0j;
          acc[2] += d * d;
          d = xb - x0j;
          acc[3] += d * d;
        }
      }
      __syncthreads();
      {
        const EvalRowsOp op(p, S);
        sweep<2, double>(p.K.rp, p.K.ci, p.K.v, bp.bk, k0, k1, r0, r1, LK, op, acc + 4, lds, red);
      }
      __syncthreads();
      {
        const EvalColsOp op(p, S);
        sweep<2, double>(p.KT.rp, p.KT.ci, p.KT.v, bp.bt, t0, t1, c0, c1, LT, op, acc + 12, lds, red);
      }
      block_sum<18>(acc, red);
      if (threadIdx.x == 0) eval_decision(S, p, tr, acc, qn0, cn0);
      __syncthreads();
      if (S->restart_flag) {
        const int cur = S->cur, cand = S->cand_avg;
        double* __restrict__ x = sel(cur, p.x[0], p.x[1]);
        for (int j = c0 + threadIdx.x; j < c1; j += kBlock) {
          const double xc = cand ? p.xbar[j] : x[j];
          x[j] = xc;
          p.x0[j] = xc;
          p.xsum[j] = 0.0;
        }
        __syncthreads();
        const RestartYOp op(p, S);
        double dummy[1];
        if (f32) sweep<1, float>(p.K.rp, p.K.ci, p.K.vf, bp.bk, k0, k1, r0, r1, LK, op, dummy, lds, red);
        else sweep<1, double>(p.K.rp, p.K.ci, p.K.v, bp.bk, k0, k1, r0, r1, LK, op, dummy, lds, red);
        __syncthreads();
        if (threadIdx.x == 0) S->restart_flag = 0;
      }
    } else {
      // --- one attempt of Algorithm 2
      double acc[3] = {0.0, 0.0, 0.0};
      {
        const PrimalOp op(p, S);
        if (f32) sweep<1, float>(p.KT.rp, p.KT.ci, p.KT.vf, bp.bt, t0, t1, c0, c1, LT, op, acc, lds, red);
        else sweep<1, double>(p.KT.rp, p.KT.ci, p.KT.v, bp.bt, t0, t1, c0, c1, LT, op, acc, lds, red);
      }
      __syncthreads();
      {
        const DualOp op(p, S);
        if (f32) sweep<1, float>(p.K.rp, p.K.ci, p.K.vf, bp.bk, k0, k1, r0, r1, LK, op, acc + 1, lds, red);
        else sweep<1, double>(p.K.rp, p.K.ci, p.K.v, bp.bk, k0, k1, r0, r1, LK, op, acc + 1, lds, red);
      }
      block_sum<3>(acc, red);
      if (threadIdx.x == 0) {
        step_decision(S, p, tr, acc[0], acc[1], acc[2]);
        rejected = S->k == k_seen ? rejected + 1 : 0;
        k_seen = S->k;
        if (!S->done && rejected >= bp.max_reject) {
          S->status = 4;
          S->ret_avg = 0;
          S->done = 1;
        }
      }
    }
    if (threadIdx.x == 0 && !S->done && bp.ticks && wall_clock64() - *bp.t0 > bp.ticks) {
      S->status = 3;
      S->ret_avg = 0;
      S->done = 1;
    }
    __syncthreads();
    if (S->done) break;
  }
  // --- output of this LP (as the output op and k_output_y)
  {
    const OutputOp op(p, S);
    double dummy[1];
    sweep<1, double>(p.KT.rp, p.KT.ci, p.KT.v, bp.bt, t0, t1, c0, c1, LT, op, dummy, lds, red);
    const int cur = S->cur, ra = S->ret_avg;
    const double* __restrict__ y = ra ? p.ybar : sel(cur, p.y[0], p.y[1]);
    for (int i = r0 + threadIdx.x; i < r1; i += kBlock) {
      const double v = p.D1[i] * y[i];
      p.yo[i] = p.le[i] ? -v : v;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) bp.st[b] = *S;
}

// Persistent batch solver: every workgroup takes LPs from the queue until it
// is empty, so the launch ends when every LP has been solved.
__global__ __launch_bounds__(kBlock) void k_batch(Params p, BatchParams bp) {
  __shared__ DevState S;
  __shared__ double red[18 * (kBlock / 64)];
  __shared__ double lds[2 * kTile];
  __shared__ int slot;
  for (;;) {
    if (threadIdx.x == 0) slot = (int)atomicAdd(bp.queue, 1u);
    __syncthreads();
    const int q = slot;
    __syncthreads();
    if (q >= bp.count) break;
    batch_solve_one(p, bp, bp.order[q], &S, red, lds);
  }
}

__global__ void k_stamp(uint64_t* t0) {
  if (threadIdx.x == 0) *t0 = wall_clock64();
}

// Per-LP sums of squares of a[off[b] .. off[b+1]) in blocks of 4096 (serial
// inside a block and across blocks), one thread per LP.
__global__ void k_seg_sumsq(int nlp, const int32_t* __restrict__ off, const double* __restrict__ a,
                            double* __restrict__ out, int stride, int slot) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nlp; b += gridDim.x * blockDim.x) {
    double tot = 0.0;
    for (int64_t i0 = off[b]; i0 < off[b + 1]; i0 += 4096) {
      const int64_t i1 = i0 + 4096 < off[b + 1] ? i0 + 4096 : off[b + 1];
      double s = 0.0;
      for (int64_t i = i0; i < i1; ++i) s = __dadd_rn(s, __dmul_rn(a[i], a[i]));
      tot = __dadd_rn(tot, s);
    }
    out[stride * b + slot] = tot;
  }
}

// Per-LP max |K~_ij| over the LP's nonzeros.
__global__ void k_seg_absmax(int nlp, const int32_t* __restrict__ row_off, const int32_t* __restrict__ rp,
                             const double* __restrict__ v, double* __restrict__ out) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < nlp; b += gridDim.x * blockDim.x) {
    double mx = 0.0;
    for (int e = rp[row_off[b]]; e < rp[row_off[b + 1]]; ++e) {
      const double a = fabs(v[e]);
      mx = a > mx ? a : mx;
    }
    out[b] = mx;
  }
}

// ---------------------------------------------------------------------------- launchers

static inline int elem_grid(int n) {
  int g = (n + kBlock - 1) / kBlock;
  if (g > kElemBlocks) g = kElemBlocks;
  return g < 1 ? 1 : g;
}

// One pass of `Op` over its matrix in the matrix's layout.
template <class Op, typename VT>
static void launch_op(const Params& p, const DevCsr& M, hipStream_t s) {
  if (M.layout == 0) {
    hipLaunchKernelGGL((k_fused<Op, VT>), dim3(M.nblocks), dim3(kBlock), 0, s, p);
  } else {
    hipLaunchKernelGGL((k_seg<Op, VT>), dim3(M.pan.nsblocks), dim3(kBlock), 0, s, p);
    hipLaunchKernelGGL((k_rows<Op>), dim3(M.rows_grid), dim3(kBlock), 0, s, p);
  }
}

void launch_primal(const Params& p, hipStream_t s) {
  if (p.use_f32) launch_op<PrimalOp, float>(p, p.KT, s);
  else launch_op<PrimalOp, double>(p, p.KT, s);
}

void launch_dual(const Params& p, hipStream_t s) {
  if (p.use_f32) launch_op<DualOp, float>(p, p.K, s);
  else launch_op<DualOp, double>(p, p.K, s);
}

void launch_decide(const Params& p, hipStream_t s) {
  hipLaunchKernelGGL(k_decide, dim3(1), dim3(kDecideBlock), 0, s, p);
}

void launch_eval(const Params& p, hipStream_t s) {
  const int ge = elem_grid(p.n);
  hipLaunchKernelGGL(k_eval_x, dim3(ge), dim3(kBlock), 0, s, p);
  launch_op<EvalRowsOp, double>(p, p.K, s);
  launch_op<EvalColsOp, double>(p, p.KT, s);
  hipLaunchKernelGGL(k_eval_decide, dim3(1), dim3(kDecideBlock), 0, s, p, ge);
  hipLaunchKernelGGL(k_restart_x, dim3(ge), dim3(kBlock), 0, s, p);
  if (p.use_f32) launch_op<RestartYOp, float>(p, p.K, s);
  else launch_op<RestartYOp, double>(p, p.K, s);
}

void launch_init(const Params& p, const double* xs, const double* ys, hipStream_t s) {
  hipLaunchKernelGGL(k_init_x, dim3(elem_grid(p.n)), dim3(kBlock), 0, s, p, xs);
  hipLaunchKernelGGL(k_init_y, dim3(elem_grid(p.m)), dim3(kBlock), 0, s, p, ys);
}

void launch_output(const Params& p, hipStream_t s) {
  launch_op<OutputOp, double>(p, p.KT, s);
  hipLaunchKernelGGL(k_output_y, dim3(elem_grid(p.m)), dim3(kBlock), 0, s, p);
}

void launch_probe(const Params& p, int which, hipStream_t s) {
  const bool f = p.use_f32 != 0;
  if (which == 0) {
    if (f) launch_op<ProbeOp<0>, float>(p, p.K, s);
    else launch_op<ProbeOp<0>, double>(p, p.K, s);
  } else {
    if (f) launch_op<ProbeOp<1>, float>(p, p.KT, s);
    else launch_op<ProbeOp<1>, double>(p, p.KT, s);
  }
}

void launch_batch(const Params& p, const BatchParams& bp, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, s, const_cast<uint64_t*>(bp.t0));
  hipLaunchKernelGGL(k_batch, dim3(grid), dim3(kBlock), 0, s, p, bp);
}

int batch_occupancy() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch, kBlock, 0) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

void launch_seg_sumsq(int nlp, const int32_t* off, const double* a, double* out, int stride, int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_seg_sumsq, dim3((nlp + 255) / 256), dim3(256), 0, s, nlp, off, a, out, stride, slot);
}

void launch_seg_absmax(int nlp, const int32_t* row_off, const int32_t* rp, const double* v, double* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_seg_absmax, dim3((nlp + 255) / 256), dim3(256), 0, s, nlp, row_off, rp, v, out);
}

void launch_set_limit(DevState* st, int status, hipStream_t s) {
  hipLaunchKernelGGL(k_set_limit, dim3(1), dim3(1), 0, s, st, status);
}

}  // namespace pdlp
