// Hot-path kernels of restarted PDHG for LP on gfx950 (arXiv 2311.12180).
//
// Every product with K~ or K~' is a row gather over one of the two CSR copies
// (no atomics on values, so results are bitwise reproducible run to run).  A
// row block is either a run of short rows whose nonzeros (at most kTile) are
// streamed once, coalesced, into LDS as products and then summed per row by a
// power-of-two group of lanes, or one long row (more than kTile nonzeros)
// swept by the whole workgroup.  No workgroup ever waits for or reads the
// results of another workgroup of the same launch: reductions leave one
// partial per workgroup and a single-workgroup kernel after the launch adds
// them in a fixed order (so no device-scope fences inside the big kernels).
//
// The PDHG updates of eq. (pdhg) are the epilogues of the row sums:
//   k_primal : (K~'y)_j -> x'_j = proj_[l,u](x_j - (eta/omega)(c_j - (K~'y)_j)), dx_j = x'_j - x_j
//   k_dual   : (K~dx)_i -> y'_i = proj(y_i + eta*omega*(q_i - (K~x)_i - 2(K~dx)_i))
//   k_decide : the Algorithm 2 step-size decision on the reduced norms.
// Evaluation kernels form the weighted averages, eq. (kkt) for both the
// current and the average iterate and the Section 4.1 termination quantities;
// k_eval_decide takes the Section 3.4 restart decision; restart kernels apply it.
#include <math.h>

#include "pdlp_dev.h"

namespace pdlp {

constexpr int kDecideBlock = 1024;   // threads of the single-workgroup reduction kernels

// ---------------------------------------------------------------------------- helpers

template <typename T>
__device__ __forceinline__ T sel(int c, T a0, T a1) { return c ? a1 : a0; }

// Workgroups are dispatched round-robin over the 8 XCDs; with remap on, each
// XCD gets a contiguous range of row blocks (each XCD has its own L2).
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
__device__ __forceinline__ const VT* values(const DevCsr& M);
template <>
__device__ __forceinline__ const double* values<double>(const DevCsr& M) { return M.v; }
template <>
__device__ __forceinline__ const float* values<float>(const DevCsr& M) { return M.vf; }

// Row block driver: runs `epi(row, sums)` exactly once for every row of the
// block.  Short rows: the products val * gathered vector(s) are staged in LDS
// (coalesced matrix stream), then each row is summed by L lanes (L = largest
// power of two <= 64 with L * rows <= kBlock) and the group's first lane runs
// the epilogue.  A long row: the workgroup sweeps it with a stride of kBlock,
// reduces, and thread 0 runs the epilogue.
template <int NV, typename VT, class G, class E>
__device__ __forceinline__ void spmv_block(const DevCsr& M, const RowBlock& rb, double* __restrict__ lds,
                                           double* red, G&& gather, E&& epi) {
  const VT* __restrict__ v = values<VT>(M);
  const int32_t* __restrict__ rp = M.rp;
  const int32_t* __restrict__ ci = M.ci;
  const int r0 = rb.r0, r1 = rb.r1;
  const int e0 = rp[r0];
  const int ne = rp[r1] - e0;
  if (ne > kTile) {
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
    for (int e = e0 + (int)threadIdx.x; e < e0 + ne; e += kBlock) {
      const double a = (double)v[e];
      double g[NV];
      gather(ci[e], g);
#pragma unroll
      for (int k = 0; k < NV; ++k) s[k] += a * g[k];
    }
    block_sum<NV>(s, red);
    if (threadIdx.x == 0) epi(r0, s);
    return;
  }
  for (int e = threadIdx.x; e < ne; e += kBlock) {
    const double a = (double)v[e0 + e];
    double g[NV];
    gather(ci[e0 + e], g);
#pragma unroll
    for (int k = 0; k < NV; ++k) lds[k * kTile + e] = a * g[k];
  }
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

// ---------------------------------------------------------------------------- PDHG step

// Primal step fused with the K~' product, one pass over the rows of K~'.
// Also adds the previously accepted x to the running weighted sum.
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_primal(Params p) {
  __shared__ double lds[kTile];
  __shared__ double red[4];
  const DevState* st = p.st;
  if (attempt_idle(st)) return;
  const int cur = st->cur;
  const double eta = st->eta, omega = st->omega;
  const double tau = eta / omega;
  const int pend = st->has_pending;
  const double pw = st->pending_w;
  const double* __restrict__ y = sel(cur, p.y[0], p.y[1]);
  const double* __restrict__ x = sel(cur, p.x[0], p.x[1]);
  double* __restrict__ xn = sel(cur, p.x[1], p.x[0]);
  double* __restrict__ dx = p.dx;
  double* __restrict__ xsum = p.xsum;
  const double* __restrict__ c = p.c;
  const double* __restrict__ lo = p.l;
  const double* __restrict__ hi = p.u;
  const int b = logical_block(p.KT.nblocks, p.xcd_remap);
  const RowBlock rb = p.KT.blocks[b];
  double acc[1] = {0.0};
  spmv_block<1, VT>(
      p.KT, rb, lds, red, [&](int i, double* g) { g[0] = y[i]; },
      [&](int j, const double* s) {
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
      });
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) p.partA[b] = acc[0];
}

// Dual step fused with the K~ product, one pass over the rows of K~.  It
// gathers dx = x' - x (written by the primal kernel), so K~dx, and with it the
// step bound's denominator dy'K~dx, is a direct product rather than the
// difference of two nearly equal products.
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_dual(Params p) {
  __shared__ double lds[kTile];
  __shared__ double red[2 * 4];
  const DevState* st = p.st;
  if (attempt_idle(st)) return;
  const int cur = st->cur;
  const double sigma = st->eta * st->omega;
  const int pend = st->has_pending;
  const double pw = st->pending_w;
  const double* __restrict__ dx = p.dx;
  const double* __restrict__ y = sel(cur, p.y[0], p.y[1]);
  double* __restrict__ yn = sel(cur, p.y[1], p.y[0]);
  const double* __restrict__ kx = sel(cur, p.kx[0], p.kx[1]);
  double* __restrict__ kxn = sel(cur, p.kx[1], p.kx[0]);
  double* __restrict__ ysum = p.ysum;
  const double* __restrict__ q = p.q;
  const int8_t* __restrict__ ineq = p.ineq;
  const int b = logical_block(p.K.nblocks, p.xcd_remap);
  const RowBlock rb = p.K.blocks[b];
  double acc[2] = {0.0, 0.0};
  spmv_block<1, VT>(
      p.K, rb, lds, red, [&](int j, double* g) { g[0] = dx[j]; },
      [&](int i, const double* s) {
        // s[0] = (K~ dx)_i; K~(2x' - x) = K~x + 2 K~dx and K~x' = K~x + K~dx
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
      });
  block_sum<2>(acc, red);
  if (threadIdx.x == 0) {
    p.partB[2 * b] = acc[0];
    p.partB[2 * b + 1] = acc[1];
  }
}

// Algorithm 2 decision on the reduced norms (single workgroup): eta_bar =
// (omega ||dx||^2 + ||dy||^2 / omega) / (2 |dy'K dx|), eta' = min((1 - (k+2)^-0.3)
// eta_bar, (1 + (k+2)^-0.6) eta); accept when eta <= eta_bar.  It also clears
// the restart flag of the previous evaluation (its restart kernels have run).
__global__ __launch_bounds__(kDecideBlock) void k_decide(Params p) {
  __shared__ double red[3 * (kDecideBlock / 64)];
  DevState* st = p.st;
  if (threadIdx.x == 0 && st->restart_flag) st->restart_flag = 0;
  if (attempt_idle(st)) return;
  double r[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < p.KT.nblocks; i += kDecideBlock) r[0] += p.partA[i];
  for (int i = threadIdx.x; i < p.K.nblocks; i += kDecideBlock) {
    r[1] += p.partB[2 * i];
    r[2] += p.partB[2 * i + 1];
  }
  block_sum<3, kDecideBlock / 64>(r, red);
  if (threadIdx.x != 0) return;
  const double nx = r[0], ny = r[1], dyk = r[2];
  const double eta = st->eta, omega = st->omega;
  const double num = omega * nx + ny / omega;
  const double den = 2.0 * fabs(dyk);
  const double eta_bar = den > 0.0 ? num / den : INFINITY;
  const double kk = (double)(st->k + 2);
  const double a = (1.0 - pow(kk, -0.3)) * eta_bar;
  const double bb = (1.0 + pow(kk, -0.6)) * eta;
  const double eta_next = a < bb ? a : bb;
  const int acc = eta <= eta_bar;
  if (st->n_att < p.tr.cap) {
    const int64_t s = st->n_att++;
    p.tr.att_k[s] = st->k;
    p.tr.att_eta[s] = eta;
    p.tr.att_etabar[s] = eta_bar;
    p.tr.att_acc[s] = (int8_t)acc;
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

// ---------------------------------------------------------------------------- evaluation

__device__ __forceinline__ bool eval_idle(const DevState* st) { return st->done | !st->need_eval; }

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

// Rows of K~: K~x and K~x_bar (FP64 matrix), the primal residual of eq. (kkt)
// (scaled, and unscaled by D1^-1 for Section 4.1), q'y, q'y_bar, and the
// y-space part of the averages.
__global__ __launch_bounds__(kBlock) void k_eval_rows(Params p) {
  __shared__ double lds[2 * kTile];
  __shared__ double red[8 * 4];
  const DevState* st = p.st;
  if (eval_idle(st)) return;
  const int cur = st->cur, init = st->initial, pend = st->has_pending;
  const double pw = st->pending_w, se = st->sum_eta;
  const double* __restrict__ x = sel(cur, p.x[0], p.x[1]);
  const double* __restrict__ xb = p.xbar;
  const double* __restrict__ y = sel(cur, p.y[0], p.y[1]);
  const int b = logical_block(p.K.nblocks, p.xcd_remap);
  const RowBlock rb = p.K.blocks[b];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  spmv_block<2, double>(
      p.K, rb, lds, red,
      [&](int j, double* g) {
        g[0] = x[j];
        g[1] = xb[j];
      },
      [&](int i, const double* s) {
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
      });
  block_sum<8>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 8; ++k) p.partE1[8 * b + k] = acc[k];
  }
}

// Rows of K~': K~'y and K~'y_bar (FP64 matrix), lambda = proj_Lambda(c - K~'y),
// the dual residual (scaled, and unscaled by D2^-1), l'lambda+ - u'lambda-.
__global__ __launch_bounds__(kBlock) void k_eval_cols(Params p) {
  __shared__ double lds[2 * kTile];
  __shared__ double red[6 * 4];
  const DevState* st = p.st;
  if (eval_idle(st)) return;
  const int cur = st->cur;
  const double* __restrict__ y = sel(cur, p.y[0], p.y[1]);
  const double* __restrict__ yb = p.ybar;
  const int b = logical_block(p.KT.nblocks, p.xcd_remap);
  const RowBlock rb = p.KT.blocks[b];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  spmv_block<2, double>(
      p.KT, rb, lds, red,
      [&](int i, double* g) {
        g[0] = y[i];
        g[1] = yb[i];
      },
      [&](int j, const double* s) {
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
      });
  block_sum<6>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) p.partE2[6 * b + k] = acc[k];
  }
}

// Reduce every evaluation partial (single workgroup, fixed order) and decide:
// termination (Section 4.1) on both iterates, else the restart candidate and
// the restart criteria (Section 3.4), the primal weight update (Section 2.2).
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
  for (int i = threadIdx.x; i < p.K.nblocks; i += kDecideBlock) {
#pragma unroll
    for (int k = 0; k < 8; ++k) S[4 + k] += p.partE1[8 * i + k];
  }
  for (int i = threadIdx.x; i < p.KT.nblocks; i += kDecideBlock) {
#pragma unroll
    for (int k = 0; k < 6; ++k) S[12 + k] += p.partE2[6 * i + k];
  }
  block_sum<18, kDecideBlock / 64>(S, red);
  if (threadIdx.x != 0) return;
  // S: 0 c'x 1 c'xb 2 |x-x0|^2 3 |xb-x0|^2 | 4,5 rp2 scaled 6,7 rp2 unscaled 8,9 q'y 10,11 |y-y0|^2
  //    | 12,13 rd2 scaled 14,15 rd2 unscaled 16,17 l'lam+ - u'lam-     (pairs: current, average)
  const double omega = st->omega;
  double pobj[2], dobj[2], rel[2], rg[2], rpr[2], rdr[2];
  for (int it = 0; it < 2; ++it) {
    pobj[it] = S[0 + it];
    dobj[it] = S[8 + it] + S[16 + it];
    rg[it] = fabs(dobj[it] - pobj[it]) / (1.0 + fabs(dobj[it]) + fabs(pobj[it]));
    rpr[it] = sqrt(S[6 + it]) / (1.0 + p.qnorm0);
    rdr[it] = sqrt(S[14 + it]) / (1.0 + p.cnorm0);
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
  if (st->n_eval < p.tr.cap) {
    const int64_t s = st->n_eval++;
    p.tr.ev_k[s] = st->k;
    p.tr.ev_kkt_cur[s] = kc_cur;
    p.tr.ev_kkt_avg[s] = kc_avg;
    p.tr.ev_cand[s] = (int8_t)cand;
    p.tr.ev_reason[s] = (int8_t)reason;
    p.tr.ev_omega[s] = om;
  }
}

// ---------------------------------------------------------------------------- restart

// x-space part of a restart: z^{n+1,0} = candidate, sums cleared.
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

// y-space part of a restart, plus K~x of the new x (in the precision of the
// steps).  The flag is cleared by the next k_decide.
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_restart_y(Params p) {
  __shared__ double lds[kTile];
  __shared__ double red[4];
  const DevState* st = p.st;
  if (!st->restart_flag) return;
  const int cur = st->cur, cand = st->cand_avg;
  const double* __restrict__ x = sel(cur, p.x[0], p.x[1]);
  double* __restrict__ y = sel(cur, p.y[0], p.y[1]);
  double* __restrict__ kx = sel(cur, p.kx[0], p.kx[1]);
  const int b = logical_block(p.K.nblocks, p.xcd_remap);
  const RowBlock rb = p.K.blocks[b];
  spmv_block<1, VT>(
      p.K, rb, lds, red, [&](int j, double* g) { g[0] = x[j]; },
      [&](int i, const double* s) {
        const double yc = cand ? p.ybar[i] : y[i];
        y[i] = yc;
        p.y0[i] = yc;
        p.ysum[i] = 0.0;
        kx[i] = s[0];
      });
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

__global__ __launch_bounds__(kBlock) void k_init_y(Params p, const double* __restrict__ ys,
                                                   const int8_t* __restrict__ le) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < p.m; i += gridDim.x * kBlock) {
    double v = 0.0;
    if (ys) {
      v = (le[i] ? -ys[i] : ys[i]) / p.D1[i];
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

// Output over the rows of K~': x = D2 x~, lambda = D2^-1 proj_Lambda(c~ - K~'y~).
__global__ __launch_bounds__(kBlock) void k_output_cols(Params p, double* __restrict__ xo,
                                                        double* __restrict__ rco) {
  __shared__ double lds[kTile];
  __shared__ double red[4];
  const DevState* st = p.st;
  const int cur = st->cur, ra = st->ret_avg;
  const double* __restrict__ x = ra ? p.xbar : sel(cur, p.x[0], p.x[1]);
  const double* __restrict__ y = ra ? p.ybar : sel(cur, p.y[0], p.y[1]);
  const int b = logical_block(p.KT.nblocks, p.xcd_remap);
  const RowBlock rb = p.KT.blocks[b];
  spmv_block<1, double>(
      p.KT, rb, lds, red, [&](int i, double* g) { g[0] = y[i]; },
      [&](int j, const double* s) {
        const double d2 = p.D2[j];
        xo[j] = d2 * x[j];
        rco[j] = proj_lambda(p.c[j] - s[0], p.l[j], p.u[j]) / d2;
      });
}

// Output of y = D1 y~, negated back on LE rows.
__global__ __launch_bounds__(kBlock) void k_output_y(Params p, double* __restrict__ yo,
                                                     const int8_t* __restrict__ le) {
  const DevState* st = p.st;
  const int cur = st->cur, ra = st->ret_avg;
  const double* __restrict__ y = ra ? p.ybar : sel(cur, p.y[0], p.y[1]);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < p.m; i += gridDim.x * kBlock) {
    const double v = p.D1[i] * y[i];
    yo[i] = le[i] ? -v : v;
  }
}

__global__ void k_set_limit(DevState* st, int status) {
  if (!st->done) {
    st->status = status;
    st->ret_avg = 0;
    st->done = 1;
  }
}

// ---------------------------------------------------------------------------- launchers

static inline int elem_grid(int n) {
  int g = (n + kBlock - 1) / kBlock;
  if (g > kElemBlocks) g = kElemBlocks;
  return g < 1 ? 1 : g;
}

void launch_primal(const Params& p, hipStream_t s) {
  if (p.use_f32) hipLaunchKernelGGL(k_primal<float>, dim3(p.KT.nblocks), dim3(kBlock), 0, s, p);
  else hipLaunchKernelGGL(k_primal<double>, dim3(p.KT.nblocks), dim3(kBlock), 0, s, p);
}

void launch_dual(const Params& p, hipStream_t s) {
  if (p.use_f32) hipLaunchKernelGGL(k_dual<float>, dim3(p.K.nblocks), dim3(kBlock), 0, s, p);
  else hipLaunchKernelGGL(k_dual<double>, dim3(p.K.nblocks), dim3(kBlock), 0, s, p);
}

void launch_decide(const Params& p, hipStream_t s) {
  hipLaunchKernelGGL(k_decide, dim3(1), dim3(kDecideBlock), 0, s, p);
}

void launch_eval(const Params& p, hipStream_t s) {
  const int ge = elem_grid(p.n);
  hipLaunchKernelGGL(k_eval_x, dim3(ge), dim3(kBlock), 0, s, p);
  hipLaunchKernelGGL(k_eval_rows, dim3(p.K.nblocks), dim3(kBlock), 0, s, p);
  hipLaunchKernelGGL(k_eval_cols, dim3(p.KT.nblocks), dim3(kBlock), 0, s, p);
  hipLaunchKernelGGL(k_eval_decide, dim3(1), dim3(kDecideBlock), 0, s, p, ge);
  hipLaunchKernelGGL(k_restart_x, dim3(ge), dim3(kBlock), 0, s, p);
  if (p.use_f32) hipLaunchKernelGGL(k_restart_y<float>, dim3(p.K.nblocks), dim3(kBlock), 0, s, p);
  else hipLaunchKernelGGL(k_restart_y<double>, dim3(p.K.nblocks), dim3(kBlock), 0, s, p);
}

void launch_init(const Params& p, const double* xs, const double* ys, const int8_t* le, hipStream_t s) {
  hipLaunchKernelGGL(k_init_x, dim3(elem_grid(p.n)), dim3(kBlock), 0, s, p, xs);
  hipLaunchKernelGGL(k_init_y, dim3(elem_grid(p.m)), dim3(kBlock), 0, s, p, ys, le);
}

void launch_output(const Params& p, double* xo, double* yo, double* rco, const int8_t* le, hipStream_t s) {
  hipLaunchKernelGGL(k_output_cols, dim3(p.KT.nblocks), dim3(kBlock), 0, s, p, xo, rco);
  hipLaunchKernelGGL(k_output_y, dim3(elem_grid(p.m)), dim3(kBlock), 0, s, p, yo, le);
}

void launch_set_limit(DevState* st, int status, hipStream_t s) {
  hipLaunchKernelGGL(k_set_limit, dim3(1), dim3(1), 0, s, st, status);
}

}  // namespace pdlp
