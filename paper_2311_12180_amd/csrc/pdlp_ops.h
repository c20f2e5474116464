// Device code shared by the single-LP kernels (kernels.hip) and the batched
// kernel (batch.hip): helpers, the LDS-tiled row-block sweep, the ops (what a
// pass over K~ or K~' gathers and what its row epilogue computes) and the
// Algorithm 2 / evaluation decisions.  Both translation units include it, so
// both paths run the same arithmetic.
#pragma once
#include <math.h>

#include "pdlp_dev.h"

namespace pdlp {

// ---------------------------------------------------------------------------- helpers

template <typename T>
__device__ __forceinline__ T sel(int c, T a0, T a1) { return c ? a1 : a0; }

// Workgroups are dispatched round-robin over the 8 XCDs; with remap on, each
// XCD gets a contiguous range of row blocks.  i is the dispatch-order index
// (blockIdx.x plus a multiple of a grid that is a multiple of 8, so that it
// stays on the same XCD).
__device__ __forceinline__ int logical_block(int i, int nb, int remap) {
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

// Buffer-resource word 3 for raw dword buffer loads on gfx9-family chips.
constexpr int kBufferWord3 = 0x00020000;
// Cache policy of the matrix stream: nt (no temporal reuse expected), so the
// stream does not push the gathered vector out of L2.
constexpr int kStreamAux = 2;

template <typename VT>
__device__ __forceinline__ double stream_value(__amdgpu_buffer_rsrc_t r, int e) {
  if constexpr (sizeof(VT) == 8)
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, e * 8, 0, kStreamAux));
  else
    return (double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, e * 4, 0, kStreamAux));
}

// Loads of one tile of nonzeros [base, base + count) (count <= TILE), for a
// workgroup of BS threads (TILE / BS nonzeros per thread): each
// thread first issues all of its column and value loads, then all of its
// gathers, so a tile costs two memory round trips per thread instead of two
// per nonzero.  f(e, a, g) receives the tile-relative index, the value and the
// NV gathered entries.  The stream is read with buffer loads on resources
// based at the tile (32-bit offsets: fewer address registers and
// instructions than 64-bit global addresses, 3 % faster step passes; the
// hardware also bounds each load by the resource's size).
template <int NV, typename VT, int BS = kBlock, int TILE = kTile, class G, class F>
__device__ __forceinline__ void tile_products(const int32_t* __restrict__ ci, const VT* __restrict__ v, int base,
                                              int count, G&& gather, F&& f) {
  constexpr int kPer = TILE / BS;
  if (count <= 0) return;
  const __amdgpu_buffer_rsrc_t rc =
      __builtin_amdgcn_make_buffer_rsrc((void*)(ci + base), 0, count * 4, kBufferWord3);
  const __amdgpu_buffer_rsrc_t rv =
      __builtin_amdgcn_make_buffer_rsrc((void*)(v + base), 0, count * (int)sizeof(VT), kBufferWord3);
  // Loads are unconditional (past the end they repeat the last entry, an
  // in-bounds index) so the loop body is straight-line code and every load of
  // the tile is in flight at once; only f is predicated.
  int col[kPer];
  double a[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = (int)threadIdx.x + u * BS;
    const int ee = e < count ? e : count - 1;
    col[u] = __builtin_amdgcn_raw_buffer_load_b32(rc, ee * 4, 0, kStreamAux);
    a[u] = stream_value<VT>(rv, ee);
  }
  double g[kPer][NV];
#pragma unroll
  for (int u = 0; u < kPer; ++u) gather(col[u], g[u]);
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = (int)threadIdx.x + u * BS;
    if (e < count) f(e, a[u], g[u]);
  }
}

// Row block driver over a CSR-like structure (rp, ci, v) for a workgroup of
// BS threads and tiles of TILE nonzeros: runs `epi(row, sums)` exactly once for
// every row of the block.  Short rows: the products val * gathered vector(s)
// are staged in LDS (coalesced matrix stream), then each row is summed by L
// lanes (L = largest power of two <= 64 with L * rows <= BS) and the group's
// first lane runs the epilogue.  A long row: the workgroup sweeps it tile by
// tile (thread t takes entries t, t + BS, ...), reduces, and thread 0 runs the
// epilogue.
// SPLIT > 1 loads a tile in SPLIT consecutive parts (fewer loads in flight per
// thread, fewer registers) without changing the tile or the sums.
// `rp` is the row-pointer array, or any object with rp[r] (an LDS copy).
template <int NV, typename VT, int BS = kBlock, int TILE = kTile, int SPLIT = 1, class RP, class G, class E>
__device__ __forceinline__ void spmv_block(const RP& rp, const int32_t* __restrict__ ci,
                                           const VT* __restrict__ v, const RowBlock& rb,
                                           double* __restrict__ lds, double* red, G&& gather, E&& epi) {
  constexpr int SUB = TILE / SPLIT;
  const int r0 = rb.r0, r1 = rb.r1;
  const int e0 = rp[r0];
  const int ne = rp[r1] - e0;
  if (ne > TILE) {
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
    for (int base = e0; base < e0 + ne; base += SUB) {
      const int cnt = min(SUB, e0 + ne - base);
      tile_products<NV, VT, BS, SUB>(ci, v, base, cnt, gather, [&](int, double a, const double* g) {
#pragma unroll
        for (int k = 0; k < NV; ++k) s[k] += a * g[k];
      });
    }
    block_sum<NV, BS / 64>(s, red);
    if (threadIdx.x == 0) epi(r0, s);
    return;
  }
  for (int h = 0; h < SPLIT; ++h) {
    const int off = h * SUB;
    tile_products<NV, VT, BS, SUB>(ci, v, e0 + off, min(SUB, ne - off), gather,
                                   [&](int e, double a, const double* g) {
#pragma unroll
                                     for (int k = 0; k < NV; ++k) lds[k * TILE + off + e] = a * g[k];
                                   });
  }
  __syncthreads();
  const int nr = r1 - r0;
  int L = 64;
  while (L > 1 && L * nr > BS) L >>= 1;
  const int groups = BS / L;
  const int grp = threadIdx.x / L, lane = threadIdx.x - grp * L;
  for (int r = grp; r < nr; r += groups) {
    const int b0 = rp[r0 + r] - e0, b1 = rp[r0 + r + 1] - e0;
    // U independent partial sums per lane (8 for one gathered vector, 4 for
    // two), so the LDS reads of a lane overlap; added pairwise in a fixed order
    constexpr int U = NV == 1 ? 8 : 4;
    double p[U][NV];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < NV; ++k) p[u][k] = 0.0;
    int e = b0 + lane;
    for (; e + (U - 1) * L < b1; e += U * L) {
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < NV; ++k) p[u][k] += lds[k * TILE + e + u * L];
    }
    for (; e < b1; e += L) {
#pragma unroll
      for (int k = 0; k < NV; ++k) p[0][k] += lds[k * TILE + e];
    }
#pragma unroll
    for (int w = U / 2; w > 0; w >>= 1)
#pragma unroll
      for (int u = 0; u < w; ++u)
#pragma unroll
        for (int k = 0; k < NV; ++k) p[u][k] += p[u + w][k];
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = p[0][k];
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
// epilogue), idle(p, st), mat(p) (which CSR copy), part(p) (its partials or
// nullptr), gather(col, g) and epi(row, s, acc).

// Primal step over the rows of K~' (x-space); adds the previously accepted x
// to the running weighted sum.
struct PrimalOp {
  static constexpr int NV = 1, NACC = 1;
  __device__ static bool idle(const Params&, const DevState* st) { return attempt_idle(st); }
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
  __device__ static bool idle(const Params&, const DevState* st) { return attempt_idle(st); }
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
  static constexpr int NV = 2, NACC = 10;
  __device__ static bool idle(const Params&, const DevState* st) { return eval_idle(st); }
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
  __device__ void epi(int i, const double* s, double* acc) const { rows(i, s[0], s[1], acc); }
  // the epilogue of row i given (K~x)_i and (K~x_bar)_i
  __device__ void rows(int i, double kx, double kxb, double* acc) const {
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
      const double kv = it ? kxb : kx;
      const double yv = it ? yb : yi;
      double r = kv - qi;
      if (ie) r = (qi - kv) > 0.0 ? (qi - kv) : 0.0;
      acc[0 + it] += r * r;
      const double ru = r / d1;
      acc[2 + it] += ru * ru;
      acc[4 + it] += qi * yv;
      const double dd = yv - y0i;
      acc[6 + it] += dd * dd;
      const double gy = qi - kv;   // the y-gradient of the normalized duality gap
      acc[8 + it] += gy * gy;
    }
    if (p.gap) {
      p.kxe[0][i] = kx;
      p.kxe[1][i] = kxb;
    }
  }
};

// The same rows of an evaluation in two passes of one gathered vector each,
// for step views that hold one vector (the LDS-staged panels): first
// K~x_bar into kxb, then K~x with the epilogue above.
struct EvalKxbOp {
  static constexpr int NV = 1, NACC = 0;
  __device__ static bool idle(const Params&, const DevState* st) { return eval_idle(st); }
  __device__ static const DevCsr& mat(const Params& p) { return p.K; }
  __device__ static double* part(const Params&) { return nullptr; }
  const double* __restrict__ xb;
  double* __restrict__ kxb;
  __device__ EvalKxbOp(const Params& p, const DevState*) : xb(p.xbar), kxb(p.kxb) {}
  __device__ void gather(int j, double* g) const { g[0] = xb[j]; }
  __device__ void epi(int i, const double* s, double*) const { kxb[i] = s[0]; }
};

struct EvalRowsKxbOp : EvalRowsOp {
  static constexpr int NV = 1, NACC = 10;
  __device__ EvalRowsKxbOp(const Params& p, const DevState* st) : EvalRowsOp(p, st) {}
  __device__ void gather(int j, double* g) const { g[0] = x[j]; }
  __device__ void epi(int i, const double* s, double* acc) const { rows(i, s[0], pp->kxb[i], acc); }
};

// Rows of K~' in an evaluation: K~'y and K~'y_bar (FP64 matrix), lambda =
// proj_Lambda(c - K~'y), the dual residual (scaled, and unscaled by D2^-1),
// l'lambda+ - u'lambda-.
struct EvalColsOp {
  static constexpr int NV = 2, NACC = 8;
  __device__ static bool idle(const Params&, const DevState* st) { return eval_idle(st); }
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
      acc[6 + it] += g * g;   // (c - K'y)^2: the x-gradient of the normalized duality gap, squared
    }
    if (p.gap) {
      p.ktye[0][j] = s[0];
      p.ktye[1][j] = s[1];
    }
  }
};

// ---- infeasibility detection (Section 2.2).  Two candidate rays per
// evaluation: the last accepted step (z minus the previous iterate, which sits
// in the other buffer) and the epoch displacement z - z^{n,0} (the normalized
// iterate without its 1/t).  Farkas' lemma is tested on the unscaled LP; the
// diagonal scalings are positive, so the projections below commute with them.

// Whether the evaluation about to be decided tests the certificates: every
// infeas_every-th evaluation after the starting point's (st->evals counts the
// earlier ones).
__device__ __forceinline__ bool infeas_due(const Params& p, const DevState* st) {
  return p.infeas && !st->initial && (st->evals + 1) % p.infeas_every == 0;
}

// Projection onto the recession cone of [l, u].
__device__ __forceinline__ double recession(double d, double l, double u) {
  const bool lf = isfinite(l), uf = isfinite(u);
  if (lf && uf) return 0.0;
  if (lf) return d > 0.0 ? d : 0.0;
  if (uf) return d < 0.0 ? d : 0.0;
  return d;
}

// Rows of K~: gathers the two primal candidates x_r (written by the x-space
// evaluation pass), forms the two dual candidates y_r (clipped at 0 on
// inequality rows; written to p.yr for the column pass and the output).  Per
// candidate: ||violation of the row cones by K x_r||^2 (unscaled: K~x_r / D1),
// q'y_r, sum |q_i y_r,i|, ||D1 y_r||^2.
struct InfeasRowsOp {
  static constexpr int NV = 2, NACC = 8;
  __device__ static bool idle(const Params& p, const DevState* st) { return eval_idle(st) || !infeas_due(p, st); }
  __device__ static const DevCsr& mat(const Params& p) { return p.K; }
  __device__ static double* part(const Params& p) { return p.partE3; }
  const Params* pp;
  const double* __restrict__ y;
  const double* __restrict__ yp;
  __device__ InfeasRowsOp(const Params& p, const DevState* st) : pp(&p) {
    const int cur = st->cur;
    y = sel(cur, p.y[0], p.y[1]);
    yp = sel(cur, p.y[1], p.y[0]);
  }
  __device__ void gather(int j, double* g) const {
    g[0] = pp->xr[0][j];
    g[1] = pp->xr[1][j];
  }
  __device__ void epi(int i, const double* s, double* acc) const {
    const Params& p = *pp;
    const double d1 = p.D1[i], qi = p.q[i], yi = y[i];
    const bool ie = p.ineq[i] != 0;
    const double base[2] = {yp[i], p.y0[i]};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const double kv = s[c] / d1;
      const double v = ie ? (kv < 0.0 ? kv : 0.0) : kv;
      acc[4 * c + 0] += v * v;
      double r = yi - base[c];
      if (ie && r < 0.0) r = 0.0;
      p.yr[c][i] = r;
      const double t = qi * r;
      acc[4 * c + 1] += t;
      acc[4 * c + 2] += fabs(t);
      const double ru = d1 * r;
      acc[4 * c + 3] += ru * ru;
    }
  }
};

// Rows of K~': gathers the dual candidates y_r.  Per candidate: g = -K'y_r
// (unscaled: -K~'y_r / D2), lam = proj_Lambda(g), ||g - lam||^2,
// l'lam+ - u'lam- and the sum of its terms' magnitudes, c'x_r, sum |c_j x_r,j|,
// ||D2 x_r||^2.
struct InfeasColsOp {
  static constexpr int NV = 2, NACC = 12;
  __device__ static bool idle(const Params& p, const DevState* st) { return eval_idle(st) || !infeas_due(p, st); }
  __device__ static const DevCsr& mat(const Params& p) { return p.KT; }
  __device__ static double* part(const Params& p) { return p.partE4; }
  const Params* pp;
  __device__ InfeasColsOp(const Params& p, const DevState*) : pp(&p) {}
  __device__ void gather(int i, double* g) const {
    g[0] = pp->yr[0][i];
    g[1] = pp->yr[1][i];
  }
  __device__ void epi(int j, const double* s, double* acc) const {
    const Params& p = *pp;
    const double d2 = p.D2[j], lj = p.l[j] * d2, uj = p.u[j] * d2, cj = p.c[j];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const double g = -s[c] / d2;
      const double lam = proj_lambda(g, lj, uj);
      const double r = g - lam;
      acc[6 * c + 0] += r * r;
      const double lp = lam > 0.0 ? lam : 0.0, lm = lam < 0.0 ? -lam : 0.0;
      const double tl = lp > 0.0 ? lj * lp : 0.0, tu = lm > 0.0 ? uj * lm : 0.0;
      acc[6 * c + 1] += tl - tu;
      acc[6 * c + 2] += fabs(tl) + fabs(tu);
      const double xr = p.xr[c][j];
      const double t = cj * xr;
      acc[6 * c + 3] += t;
      acc[6 * c + 4] += fabs(t);
      const double xu = d2 * xr;
      acc[6 * c + 5] += xu * xu;
    }
  }
};

// y-space part of a restart plus K~x of the new x (in the precision of the
// steps).  The x-space part (k_restart_x) has run before.
struct RestartYOp {
  static constexpr int NV = 1, NACC = 0;
  __device__ static bool idle(const Params&, const DevState* st) { return !st->restart_flag; }
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
// With a certificate of primal infeasibility (status 5) y~ is the dual ray and
// lambda its multipliers D2^-1 proj_Lambda(-K~'y~), scaled to the unit ray;
// with one of dual infeasibility (status 6) x is the unit primal ray.
struct OutputOp {
  static constexpr int NV = 1, NACC = 0;
  __device__ static bool idle(const Params&, const DevState*) { return false; }
  __device__ static const DevCsr& mat(const Params& p) { return p.KT; }
  __device__ static double* part(const Params&) { return nullptr; }
  const Params* pp;
  const double* __restrict__ x;
  const double* __restrict__ y;
  double xs, cs, ls;
  __device__ OutputOp(const Params& p, const DevState* st) : pp(&p) {
    const int cur = st->cur, ra = st->ret_avg;
    x = ra ? p.xbar : sel(cur, p.x[0], p.x[1]);
    y = ra ? p.ybar : sel(cur, p.y[0], p.y[1]);
    xs = 1.0;   // factor on x
    cs = 1.0;   // weight of c in lambda
    ls = 1.0;   // factor on lambda
    if (st->status == 5) {
      y = p.yr[st->ray_src];
      cs = 0.0;
      ls = st->ray_scale;
    } else if (st->status == 6) {
      x = p.xr[st->ray_src];
      xs = st->ray_scale;
    }
  }
  __device__ void gather(int i, double* g) const { g[0] = y[i]; }
  __device__ void epi(int j, const double* s, double*) const {
    const Params& p = *pp;
    const double d2 = p.D2[j];
    p.xo[j] = d2 * x[j] * xs;
    p.rco[j] = proj_lambda(cs * p.c[j] - s[0], p.l[j], p.u[j]) / d2 * ls;
  }
};


// ---------------------------------------------------------------------------- decisions

// Algorithm 2 decision on the reduced norms (one thread): eta_bar =
// (omega ||dx||^2 + ||dy||^2 / omega) / (2 |dy'K dx|), eta' = min((1 - (k+2)^-0.3)
// eta_bar, (1 + (k+2)^-0.6) eta); accept when eta <= eta_bar.
static __device__ void step_decision(DevState* st, const Params& p, const Trace& tr, double nx, double ny, double dyk) {
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

// Section 3.4 restart decision on the candidate metric values (KKT_omega or
// the normalized duality gap) of the current and the average iterate: the
// candidate, criteria (i)-(iii), the primal weight update (Section 2.2), the
// restart flag; kkt0_of(cand, new omega, value) gives the next epoch's
// reference value.
template <class K0>
static __device__ void restart_decision(DevState* st, const Params& p, const Trace& tr, double kc_cur, double kc_avg,
                                        double dx2_cur, double dx2_avg, double dy2_cur, double dy2_avg,
                                        K0&& kkt0_of) {
  const double omega = st->omega;
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
    const double dxn = sqrt(cand ? dx2_avg : dx2_cur), dyn = sqrt(cand ? dy2_avg : dy2_cur);
    if (dxn > p.eps_zero && dyn > p.eps_zero) om = exp(p.theta * log(dyn / dxn) + (1.0 - p.theta) * log(omega));
    st->omega = om;
    st->restart_flag = 1;
    st->cand_avg = cand;
    st->restarts++;
    st->t = 0;
    st->sum_eta = 0.0;
    st->kkt0 = kkt0_of(cand, om, kc);
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

// ---- normalized duality gap (restart metric 1, PDLP's; Section 3.4 names it
// as the metric the KKT error replaces).  rho_r(z) = max { L(x, yh) - L(xh, y)
// : zh in Z, ||zh - z||_omega <= r } / r on the scaled LP, ||d||_omega^2 =
// omega ||dx||^2 + ||dy||^2 / omega.  The objective is linear in d = zh - z
// with gradient g = (K'y - c, q - Kx); the maximiser is
// d(lam) = proj_{Z - z}(W^-1 g / lam), W = diag(omega, 1/omega), at the lam
// where ||d(lam)||_omega = r (||d|| does not increase with lam), or at lo when
// the ball does not bind there.  lam is bracketed between
// hi = ||W^-1 g||_omega / r (where ||d|| <= r) and lo = 1e-12 hi and narrowed
// by kGapPasses passes that each evaluate kGapPoints geometrically spaced
// values; a last pass evaluates g'd at the result.  Both candidates (current,
// average) are searched in the same passes.

// The factors of d = W^-1 g / lam for one multiplier value: x-part
// g_x / (omega lam) = g_x sx, y-part g_y omega / lam = g_y sy.
struct GapScale {
  double sx[kGapPoints], sy[kGapPoints];
  double om, iom;
  __device__ GapScale(const double* lam, double omega) : om(omega), iom(1.0 / omega) {
#pragma unroll
    for (int k = 0; k < kGapPoints; ++k) {
      sx[k] = 1.0 / (omega * lam[k]);
      sy[k] = omega / lam[k];
    }
  }
};

// Contributions of column j (x-space) to candidate C's pass sums
// (acc[k] = ||d(lam_k)||^2 part, acc[4 + k] = g'd(lam_k) part).
template <int C>
__device__ __forceinline__ void gap_col(const Params& p, const double* __restrict__ x, const GapScale& g,
                                        int j, double* acc) {
  const double xc = C ? p.xbar[j] : x[j];
  const double gx = p.ktye[C][j] - p.c[j];
  const double lo = p.l[j] - xc, hi = p.u[j] - xc;
#pragma unroll
  for (int k = 0; k < kGapPoints; ++k) {
    double d = gx * g.sx[k];
    if (d < lo) d = lo;
    if (d > hi) d = hi;
    acc[k] += g.om * (d * d);
    acc[4 + k] += gx * d;
  }
}

// Contributions of row i (y-space) to candidate C's pass sums.
template <int C>
__device__ __forceinline__ void gap_row(const Params& p, const double* __restrict__ y, const GapScale& g,
                                        int i, double* acc) {
  const double yc = C ? p.ybar[i] : y[i];
  const double gy = p.q[i] - p.kxe[C][i];
  const bool ie = p.ineq[i] != 0;
#pragma unroll
  for (int k = 0; k < kGapPoints; ++k) {
    double d = gy * g.sy[k];
    if (ie && d < -yc) d = -yc;
    acc[k] += (d * d) * g.iom;
    acc[4 + k] += gy * d;
  }
}

// One thread, after a pass: narrow each candidate's bracket (R[8c + k] =
// ||d(lam_k)||^2, R[8c + 4 + k] = g'd(lam_k)) and set the next pass's values;
// after the last pass, rho and the restart decision.
static __device__ void gap_step(DevState* st, const Params& p, const Trace& tr, const double* R) {
  const int ph = st->gap_phase;
  const bool last = ph == kGapPasses + 1;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const double r = st->gap_r[c], r2 = r * r;
    double lo = st->gap_lo[c], hi = st->gap_hi[c];
    if (last) {
      st->gap_rho[c] = st->gap_mode[c] == 2 ? 0.0 : R[8 * c + 4] / r;
      continue;
    }
    if (st->gap_mode[c] == 0) {
      if (ph == 0) {
        if (R[8 * c] <= r2) {   // the ball does not bind at lo: the multiplier is lo
          st->gap_mode[c] = 1;
          hi = lo;
        }
      } else {
        // N decreases along the points: keep N(lo) > r^2 >= N(hi)
        const double l0 = st->gap_lam[c][0], l1 = st->gap_lam[c][1], l2 = st->gap_lam[c][2],
                     l3 = st->gap_lam[c][3];
        if (R[8 * c + 0] <= r2) { hi = l0; }
        else if (R[8 * c + 1] <= r2) { lo = l0; hi = l1; }
        else if (R[8 * c + 2] <= r2) { lo = l1; hi = l2; }
        else if (R[8 * c + 3] <= r2) { lo = l2; hi = l3; }
        else { lo = l3; }
      }
    }
    st->gap_lo[c] = lo;
    st->gap_hi[c] = hi;
    if (ph == kGapPasses || st->gap_mode[c] != 0) {
#pragma unroll
      for (int k = 0; k < kGapPoints; ++k) st->gap_lam[c][k] = hi;
    } else {
      const double q = exp(log(hi / lo) / (kGapPoints + 1));
      double v = lo;
#pragma unroll
      for (int k = 0; k < kGapPoints; ++k) {
        v = v * q;
        st->gap_lam[c][k] = v;
      }
    }
  }
  if (last) {
    st->gap_active = 0;
    restart_decision(st, p, tr, st->gap_rho[0], st->gap_rho[1], st->gap_dx2[0], st->gap_dx2[1], st->gap_dy2[0],
                     st->gap_dy2[1], [](int, double, double kc) { return kc; });
    return;
  }
  st->gap_phase = ph + 1;
}

// Evaluation decision on the reduced sums S (one thread): termination
// (Section 4.1) on both iterates, else the restart candidate and the restart
// criteria (Section 3.4), the primal weight update (Section 2.2).
static __device__ void eval_decision(DevState* st, const Params& p, const Trace& tr, const double* S, double qnorm0,
                              double cnorm0) {
  // S: 0 c'x 1 c'xb 2 |x-x0|^2 3 |xb-x0|^2 | 4,5 rp2 scaled 6,7 rp2 unscaled 8,9 q'y 10,11 |y-y0|^2
  //    | 12,13 rd2 scaled 14,15 rd2 unscaled 16,17 l'lam+ - u'lam-     (pairs: current, average)
  //    | 18 + 4c: InfeasRowsOp of candidate c | 26 + 6c: InfeasColsOp of candidate c (when p.infeas)
  //    | 38,39 ||q - Kx||^2 | 40,41 ||c - K'y||^2 (the normalized duality gap's gradients)
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
    // the restart metric's reference value (normalized duality gap: +inf before the first restart)
    st->kkt0 = p.gap ? INFINITY : kkt_w(0, omega);
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
  const bool due = infeas_due(p, st);
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
  if (due) {
    // Farkas certificates: a dual ray (primal infeasibility) before a primal
    // ray (dual infeasibility), the last step before the displacement.  A ray's
    // objective must exceed eps times the magnitudes it is summed from.
    const double eps = p.eps_infeas;
    double dro[2], dres[2], dnrm[2], pro[2], pres[2], pnrm[2];
    bool dok[2], pok[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      dro[c] = S[19 + 4 * c] + S[27 + 6 * c];
      dres[c] = sqrt(S[26 + 6 * c]);
      dnrm[c] = sqrt(S[21 + 4 * c]);
      dok[c] = dro[c] > 0.0 && dro[c] > eps * (S[20 + 4 * c] + S[28 + 6 * c]) && dres[c] <= eps * dro[c];
      pro[c] = S[29 + 6 * c];
      pres[c] = sqrt(S[18 + 4 * c]);
      pnrm[c] = sqrt(S[31 + 6 * c]);
      pok[c] = pro[c] < 0.0 && -pro[c] > eps * S[30 + 6 * c] && pres[c] <= eps * -pro[c];
    }
    int kind = 0, src = 0;
    if (dok[0]) { kind = 5; src = 0; }
    else if (dok[1]) { kind = 5; src = 1; }
    else if (pok[0]) { kind = 6; src = 0; }
    else if (pok[1]) { kind = 6; src = 1; }
    if (kind) {
      // (selects rather than indexing by src, which would put the arrays in scratch)
      const bool d = kind == 5, s1 = src == 1;
      const double nrm = d ? (s1 ? dnrm[1] : dnrm[0]) : (s1 ? pnrm[1] : pnrm[0]);
      const double obj = d ? (s1 ? dro[1] : dro[0]) : (s1 ? pro[1] : pro[0]);
      const double res = d ? (s1 ? dres[1] : dres[0]) : (s1 ? pres[1] : pres[0]);
      const double sc = nrm > 0.0 ? 1.0 / nrm : 0.0;
      st->status = kind;
      st->ret_avg = 0;
      st->ray_src = src;
      st->ray_scale = sc;
      st->ray_obj = obj * sc;
      st->ray_res = res * sc;
      store(0);
      st->done = 1;
      return;
    }
  }
  if (st->k >= st->max_iter) {
    st->status = 2; st->ret_avg = avg_better; store(avg_better); st->done = 1;
    return;
  }
  store(avg_better);
  if (p.gap) {
    // normalized duality gap: set up the multiplier search of each candidate's
    // trust-region problem; the restart decision follows the passes (gap_step)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const double dx2 = S[2 + c], dy2 = S[10 + c];
      st->gap_dx2[c] = dx2;
      st->gap_dy2[c] = dy2;
      const double r = sqrt(omega * dx2 + dy2 / omega);
      const double gn2 = S[40 + c] / omega + omega * S[38 + c];
      st->gap_r[c] = r;
      st->gap_rho[c] = 0.0;
      double lo = 1.0, hi = 1.0;
      if (r > 0.0 && gn2 > 0.0) {
        hi = sqrt(gn2) / r;
        lo = hi * 1e-12;
        st->gap_mode[c] = 0;
      } else {
        st->gap_mode[c] = 2;
      }
      st->gap_lo[c] = lo;
      st->gap_hi[c] = hi;
#pragma unroll
      for (int k = 0; k < kGapPoints; ++k) st->gap_lam[c][k] = lo;
    }
    st->gap_phase = 0;
    st->gap_active = 1;
    return;
  }
  restart_decision(st, p, tr, kkt_w(0, omega), kkt_w(1, omega), S[2], S[3], S[10], S[11],
                   [&](int cand, double om, double) { return kkt_w(cand, om); });
}

}  // namespace pdlp
