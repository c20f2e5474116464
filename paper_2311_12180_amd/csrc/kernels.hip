// Hot-path kernels of restarted PDHG for LP on gfx950 (arXiv 2311.12180).
//
// Every product with K~ or K~' is a row gather over one of the two CSR copies
// (no atomics on values, so results are bitwise reproducible run to run).
// Each pass over a matrix is an "op": what is gathered per nonzero, and what
// the row epilogue does with the row sums (the PDHG updates of eq. (pdhg),
// the eq. (kkt) residuals, the restart, the output).  An op runs in the
// layout chosen per matrix by timing at create; the general two:
//   fused  : row blocks -- runs of short rows whose nonzeros (at most kTile)
//            are streamed once, coalesced, into LDS as products and summed per
//            row by a power-of-two group of lanes, or one long row swept by
//            the whole workgroup -- with the epilogue in the same kernel;
//   panels : phase 1 sums the (row, column-panel) segments with workgroup i
//            serving panel i % 8 only (one XCD per panel, so the gathered
//            slice of the vector stays in that XCD's L2), phase 2 adds each
//            row's segment sums in panel order and runs the epilogue.
// The step passes may also take an LDS-staged panel layout (long rows; with
// the FP64 matrix the evaluation's rows of K~ then run on it too, as two
// passes of one gathered vector), and the passes over a matrix a SELL-64
// layout (one row per lane), both described at their kernels.
// No workgroup reads another workgroup's results inside a launch: reductions
// leave one partial per workgroup and a single-workgroup kernel after the
// launch adds them in a fixed order.
//
//   primal op (rows of K~') : x'_j = proj_[l,u](x_j - (eta/omega)(c_j - (K~'y)_j)), dx_j = x'_j - x_j
//   dual op   (rows of K~)  : y'_i = proj(y_i + eta*omega*(q_i - (K~x)_i - 2(K~dx)_i))
//   k_decide                : the Algorithm 2 step-size decision on the reduced norms
//   eval ops, k_eval_decide : averages, eq. (kkt) on current and average iterate,
//                             Section 4.1 termination, Section 2.2 infeasibility
//                             certificates, Section 3.4 restart decision
//   restart ops             : apply the restart (new z^{n+1,0}, K~x)
#include <hip/hip_ext.h>
#include <math.h>

#include "pdlp_ops.h"

namespace pdlp {

constexpr int kDecideBlock = 1024;   // threads of the single-workgroup reduction kernels

// ---------------------------------------------------------------------------- generic passes

template <class Op>
struct AccSize {
  static constexpr int N = Op::NACC > 0 ? Op::NACC : 1;
  static constexpr int RED = (Op::NACC > Op::NV ? Op::NACC : Op::NV) * (kBlock / 64);
};

// Fused layout: row blocks, epilogue in the same kernel.  TILE is the
// matrix's tiling (the blocks hold at most TILE nonzeros, or one long row).
template <class Op, typename VT, int TILE = kTile>
__global__ __launch_bounds__(kBlock) void k_fused(Params p) {
  __shared__ double lds[Op::NV * TILE];
  __shared__ double red[AccSize<Op>::RED];
  if (Op::idle(p, p.st)) return;
  const Op op(p, p.st);
  const DevCsr& M = Op::mat(p);
  // one block per workgroup, or a persistent grid striding over the blocks;
  // the partials stay one per block either way
  for (int i = blockIdx.x; i < M.nblocks; i += gridDim.x) {
    const int b = logical_block(i, M.nblocks, M.remap);
    double acc[AccSize<Op>::N];
#pragma unroll
    for (int k = 0; k < AccSize<Op>::N; ++k) acc[k] = 0.0;
    spmv_block<Op::NV, VT, kBlock, TILE>(
        M.rp, M.ci, pick<VT>(M.v, M.vf), M.blocks[b], lds, red, [&](int c, double* g) { op.gather(c, g); },
        [&](int r, const double* s) { op.epi(r, s, acc); });
    if constexpr (Op::NACC > 0) {
      block_sum<Op::NACC>(acc, red);
      if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < Op::NACC; ++k) Op::part(p)[Op::NACC * b + k] = acc[k];
      }
    }
    __syncthreads();   // the next block reuses lds
  }
}

// Panel layout, phase 1: segment sums of the blocks of panel blockIdx % 8.
template <class Op, typename VT, int TILE = kTile>
__global__ __launch_bounds__(kBlock) void k_seg(Params p) {
  __shared__ double lds[Op::NV * TILE];
  __shared__ double red[Op::NV * (kBlock / 64)];
  if (Op::idle(p, p.st)) return;
  const Op op(p, p.st);
  const PanelCsr& S = Op::mat(p).pan;
  double* __restrict__ part = S.part;
  for (int i = blockIdx.x; i < S.nsblocks; i += gridDim.x) {
    spmv_block<Op::NV, VT, kBlock, TILE>(
        S.seg_ptr, S.pci, pick<VT>(S.pv, S.pvf), S.sblocks[i], lds, red,
        [&](int c, double* g) { op.gather(c, g); },
        [&](int s, const double* sums) {
#pragma unroll
          for (int k = 0; k < Op::NV; ++k) part[Op::NV * s + k] = sums[k];
        });
    __syncthreads();   // the next block reuses lds
  }
}

// Panel layout, phase 2: each row adds its segment sums in panel order and
// runs the epilogue; one reduction partial per workgroup of a fixed grid.
template <class Op>
__global__ __launch_bounds__(kBlock) void k_rows(Params p) {
  __shared__ double red[AccSize<Op>::RED];
  if (Op::idle(p, p.st)) return;
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
      const int g = S.slot_seg[q];
#pragma unroll
      for (int k = 0; k < Op::NV; ++k) s[k] += S.part[Op::NV * g + k];
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

// LDS-staged panels, phase 1 (step passes: one gathered vector).  A work item
// is a run of one column panel's chunks: the workgroup copies the panel's
// slice of the gathered vector into LDS once; then each wavefront takes whole
// chunks, every lane summing its segment in stored order (coalesced loads of
// the lane-interleaved entries, every gather an LDS read, no barrier), and
// stores the segment sums.  A chunk's descriptor is read while the previous
// chunk is summed.
//
// After its work items, each workgroup sums blocks of the short rows' column
// panels (the step view's PanelCsr): workgroup w takes blocks w, w + grid,
// ..., with a grid that is a multiple of 8, so block j (which serves panel
// j % 8) stays on XCD j % 8, whose L2 holds that panel's slice of the vector.
// Work items finish at different times, so this latency-bound work overlaps
// other workgroups' streaming instead of following it in a launch of its own.
template <class Op, typename VT, int BS>
__global__ __launch_bounds__(BS) void k_stage(Params p) {
  static_assert(Op::NV == 1, "staged panels hold one gathered vector");
  static_assert(kTile <= kStageWidth, "a short-row block's products fit the LDS slice");
  __shared__ double xs[kStageWidth];
  __shared__ double red[BS / 64];
  if (Op::idle(p, p.st)) return;
  const Op op(p, p.st);
  const DevCsr& M = Op::mat(p);
  const StagedCsr& S = M.stg;
  double* __restrict__ part = S.part;
  const VT* __restrict__ vals = pick<VT>(S.pv, S.pvf);
  const uint16_t* __restrict__ pci = S.pci;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));   // wave-uniform: scalar chunk loop
  constexpr int kWaves = BS / 64;
  constexpr int kU = 8;   // loads in flight per lane
  for (int w = blockIdx.x; w < S.nwork; w += gridDim.x) {
    if (S.wchunk[2 * w] == S.wchunk[2 * w + 1]) continue;   // a pad slot
    const int pan = S.wpanel[w];
    const int c0 = pan * kStageWidth;
    const int nc = min(kStageWidth, S.ncols - c0);
    for (int j0 = 0; j0 < nc; j0 += kU * BS) {
      double g[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int j = j0 + u * BS + (int)threadIdx.x;
        op.gather(c0 + (j < nc ? j : nc - 1), &g[u]);
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int j = j0 + u * BS + (int)threadIdx.x;
        if (j < nc) xs[j] = g[u];
      }
    }
    __syncthreads();
    const int ch1 = S.wchunk[2 * w + 1];
    int c = S.wchunk[2 * w] + wv;
    int len = 0, off = 0, s0 = 0, s1 = 0, row = 0;
    if (c < ch1) {
      len = S.clen[c];
      off = S.coff[c];
      s0 = S.cseg[c];
      s1 = S.cseg[c + 1];
      if (s0 + lane < s1) row = S.srow[s0 + lane];
    }
    while (c < ch1) {
      const int cn = c + kWaves;
      int nlen = 0, noff = 0, ns0 = 0, ns1 = 0, nrow = 0;
      if (cn < ch1) {
        nlen = S.clen[cn];
        noff = S.coff[cn];
        ns0 = S.cseg[cn];
        ns1 = S.cseg[cn + 1];
        if (ns0 + lane < ns1) nrow = S.srow[ns0 + lane];
      }
      const int base = off + lane;
      double acc = 0.0;
      for (int k = 0; k < len; k += kU) {
        // (len is wave-uniform: the guards are scalar branches, no load past the end)
        // (values kept as loaded and widened in the sum: a conversion next to
        // its load would make each guarded load wait for itself)
        int col[kU];
        VT a[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u)
          if (k + u < len) {
            col[u] = __builtin_nontemporal_load(pci + base + (k + u) * kStageLanes);
            a[u] = __builtin_nontemporal_load(vals + base + (k + u) * kStageLanes);
          }
#pragma unroll
        for (int u = 0; u < kU; ++u)
          if (k + u < len) acc += (double)a[u] * xs[col[u]];
      }
      if (s0 + lane < s1) part[(size_t)pan * S.rlong + row] = acc;
      c = cn;
      len = nlen;
      off = noff;
      s0 = ns0;
      s1 = ns1;
      row = nrow;
    }
    __syncthreads();   // the next work item rewrites xs
  }
  // the short rows' panel blocks (products staged in xs, as in k_seg)
  const PanelCsr& Q = M.pan;
  for (int i = blockIdx.x; i < Q.nsblocks; i += gridDim.x) {
    spmv_block<1, VT, BS, kTile>(
        Q.seg_ptr, Q.pci, pick<VT>(Q.pv, Q.pvf), Q.sblocks[i], xs, red,
        [&](int col, double* g) { op.gather(col, g); }, [&](int sg, const double* sums) { Q.part[sg] = sums[0]; });
    __syncthreads();   // the next block reuses xs
  }
}

// LDS-staged panels, phase 2: workgroups [0, nrblocks) take the short rows,
// a thread per row adding the row's sums from the step view's column panels
// in panel order (a row of one nonzero takes its product directly: equal
// lengths are numbered by first column, so these gathers run in address
// order); the last nlong_groups take 64 long rows at a time, each row's
// segment sums added in four interleaved panel groups and then in group order
// (consecutive lanes read consecutive entries).  Every row runs the epilogue.
// One reduction partial per workgroup.
template <class Op, typename VT>
__global__ __launch_bounds__(kBlock) void k_stage_rows(Params p) {
  __shared__ double red[AccSize<Op>::RED];
  if (Op::idle(p, p.st)) return;
  const Op op(p, p.st);
  const DevCsr& M = Op::mat(p);
  const StagedCsr& S = M.stg;
  double acc[AccSize<Op>::N];
#pragma unroll
  for (int k = 0; k < AccSize<Op>::N; ++k) acc[k] = 0.0;
  const int nlg = S.nlong_groups, nrb = S.nrblocks;
  if ((int)blockIdx.x >= nrb) {
    // 64 long rows per workgroup: wavefront g sums panels g, g + 4, ... of
    // lane l's row (eight loads in flight), then the four sums are added in
    // wavefront order
    __shared__ double lred[kBlock / 64][64];
    constexpr int kG = kBlock / 64;
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    for (int r0 = (blockIdx.x - nrb) * 64; r0 < S.rlong; r0 += nlg * 64) {
      const int r = r0 + lane;
      double sum = 0.0;
      if (r < S.rlong) {
        const double* __restrict__ col = S.part + r;
        int q = grp;
        for (; q + 7 * kG < S.npan; q += 8 * kG) {
          double v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) v[u] = col[(size_t)(q + u * kG) * S.rlong];
#pragma unroll
          for (int u = 0; u < 8; ++u) sum += v[u];
        }
        for (; q < S.npan; q += kG) sum += col[(size_t)q * S.rlong];
      }
      lred[grp][lane] = sum;
      __syncthreads();
      if (grp == 0 && r < S.rlong) {
        double t = lred[0][lane];
#pragma unroll
        for (int g2 = 1; g2 < kG; ++g2) t += lred[g2][lane];
        op.epi(r, &t, acc);
      }
      __syncthreads();
    }
  } else {
    const PanelCsr& Q = M.pan;
    const VT* __restrict__ vals = pick<VT>(M.v, M.vf);
    for (int r = S.rlong + blockIdx.x * kBlock + (int)threadIdx.x; r < M.nrows; r += nrb * kBlock) {
      const int b = M.rp[r], e = M.rp[r + 1];
      double sum = 0.0;
      if (e - b <= 1) {
        if (e > b) {
          double g;
          op.gather(__builtin_nontemporal_load(M.ci + b), &g);
          sum = (double)__builtin_nontemporal_load(vals + b) * g;
        }
      } else {
        for (int q = Q.row_seg[r]; q < Q.row_seg[r + 1]; ++q) sum += Q.part[Q.slot_seg[q]];
      }
      op.epi(r, &sum, acc);
    }
  }
  if constexpr (Op::NACC > 0) {
    block_sum<Op::NACC>(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < Op::NACC; ++k) Op::part(p)[Op::NACC * blockIdx.x + k] = acc[k];
    }
  }
}

// SELL-64 pass (layout 4) on a persistent grid: wavefront w of the grid
// takes chunks w, w + (waves of the grid), ...; each lane sums its row's
// entries in stored order (coalesced loads of the lane-interleaved entries,
// kU of them in flight, nontemporal: the matrix is read once per pass, and
// kept out of the caches it leaves them to the vectors) and runs the
// epilogue.  With HOT, the workgroup first
// copies the leading entries of the NV gathered vectors into LDS (kSellHot / NV
// of each, at most S.hot), and gathers below that read the copy.  One
// reduction partial per workgroup.
template <class Op, typename VT, int BS, bool HOT>
__global__ __launch_bounds__(BS) void k_sell(Params p) {
  constexpr int NV = Op::NV;
  constexpr int kWaves = BS / 64;
  constexpr int kU = 8;
  constexpr int kHot = kSellHot / NV;
  __shared__ double xs[HOT ? kSellHot : 1];
  __shared__ double red[AccSize<Op>::N * kWaves];
  if (Op::idle(p, p.st)) return;
  const Op op(p, p.st);
  const DevCsr& M = Op::mat(p);
  const SellCsr& S = M.sel;
  const int hot = HOT ? min(S.hot, kHot) : 0;
  if (HOT) {
    for (int j0 = 0; j0 < hot; j0 += kU * BS) {
      double g[kU][NV];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int j = j0 + u * BS + (int)threadIdx.x;
        op.gather(j < hot ? j : hot - 1, g[u]);
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int j = j0 + u * BS + (int)threadIdx.x;
        if (j < hot) {
#pragma unroll
          for (int k = 0; k < NV; ++k) xs[k * kHot + j] = g[u][k];
        }
      }
    }
    __syncthreads();
  }
  const VT* __restrict__ vals = pick<VT>(S.sv, S.svf);
  const int32_t* __restrict__ sci = S.sci;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  double acc[AccSize<Op>::N];
#pragma unroll
  for (int k = 0; k < AccSize<Op>::N; ++k) acc[k] = 0.0;
  for (int c = blockIdx.x * kWaves + wv; c < S.nchunks; c += gridDim.x * kWaves) {
    const int len = S.clen[c];
    const int base = S.coff[c] + lane;
    double sum[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) sum[k] = 0.0;
    for (int k0 = 0; k0 < len; k0 += kU) {
      int col[kU];
      VT a[kU];   // widened in the sum (see k_stage)
      double g[kU][NV];
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (k0 + u < len) {
          col[u] = __builtin_nontemporal_load(sci + base + (k0 + u) * 64);
          a[u] = __builtin_nontemporal_load(vals + base + (k0 + u) * 64);
        }
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (k0 + u < len) {
          if (HOT && col[u] < hot) {
#pragma unroll
            for (int k = 0; k < NV; ++k) g[u][k] = xs[k * kHot + col[u]];
          } else {
            op.gather(col[u], g[u]);
          }
        }
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (k0 + u < len) {
#pragma unroll
          for (int k = 0; k < NV; ++k) sum[k] += (double)a[u] * g[u][k];
        }
    }
    const int r = c * 64 + lane;
    if (r < M.nrows) op.epi(r, sum, acc);
  }
  if constexpr (Op::NACC > 0) {
    block_sum<Op::NACC, kWaves>(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < Op::NACC; ++k) Op::part(p)[Op::NACC * blockIdx.x + k] = acc[k];
    }
  }
}

// ---------------------------------------------------------------------------- decisions


// Single-workgroup reduction of the step partials and the decision.  It also
// clears the restart flag of the previous evaluation (its restart kernels have run).
__global__ __launch_bounds__(kDecideBlock) void k_decide(Params p) {
  __shared__ double red[3 * (kDecideBlock / 64)];
  DevState* st = p.st;
  if (threadIdx.x == 0 && st->restart_flag) st->restart_flag = 0;
  if (attempt_idle(st)) return;
  double r[3] = {0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < p.KTs.nred; i += kDecideBlock) r[0] += p.partA[i];
  for (int i = threadIdx.x; i < p.Ks.nred; i += kDecideBlock) {
    r[1] += p.partB[2 * i];
    r[2] += p.partB[2 * i + 1];
  }
  block_sum<3, kDecideBlock / 64>(r, red);
  if (threadIdx.x == 0) step_decision(st, p, p.tr, r[0], r[1], r[2]);
}

// x-space part of the evaluation: flush the pending weight into the sum,
// form x_bar = sum / sum_eta, and reduce c'x, c'x_bar, ||x - x0||^2, ||x_bar - x0||^2.
__global__ __launch_bounds__(kBlock) void k_eval_x(Params p) {
  __shared__ double red[4 * (kBlock / 64)];
  const DevState* st = p.st;
  if (eval_idle(st)) return;
  const int cur = st->cur, init = st->initial, pend = st->has_pending;
  const double pw = st->pending_w, se = st->sum_eta;
  const double* __restrict__ x = sel(cur, p.x[0], p.x[1]);
  const double* __restrict__ xp = sel(cur, p.x[1], p.x[0]);
  const bool rays = infeas_due(p, st);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int j = p.col_base + blockIdx.x * kBlock + threadIdx.x; j < p.col_base + p.n; j += gridDim.x * kBlock) {
    const double xj = x[j];
    if (rays) {   // the primal candidate rays of the infeasibility test
      const double lj = p.l[j], uj = p.u[j];
      p.xr[0][j] = recession(xj - xp[j], lj, uj);
      p.xr[1][j] = recession(xj - p.x0[j], lj, uj);
    }
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


// Single-workgroup reduction of every evaluation partial in a fixed order,
// then the evaluation decision.
__global__ __launch_bounds__(kDecideBlock) void k_eval_decide(Params p, int n_e0_blocks, int n_e1) {
  __shared__ double red[22 * (kDecideBlock / 64)];
  __shared__ double E[42];
  DevState* st = p.st;
  if (eval_idle(st)) return;
  {
    double S[22];
#pragma unroll
    for (int k = 0; k < 22; ++k) S[k] = 0.0;
    for (int i = threadIdx.x; i < n_e0_blocks; i += kDecideBlock) {
#pragma unroll
      for (int k = 0; k < 4; ++k) S[k] += p.partE0[4 * i + k];
    }
    for (int i = threadIdx.x; i < n_e1; i += kDecideBlock) {
#pragma unroll
      for (int k = 0; k < 10; ++k) S[4 + k] += p.partE1[10 * i + k];
    }
    for (int i = threadIdx.x; i < p.KT.nred; i += kDecideBlock) {
#pragma unroll
      for (int k = 0; k < 8; ++k) S[14 + k] += p.partE2[8 * i + k];
    }
    block_sum<22, kDecideBlock / 64>(S, red);
    // partials order: rows 8 + 2 (gap), columns 6 + 2 (gap); E keeps the gap sums at 38..41
    if (threadIdx.x == 0) {
      for (int k = 0; k < 12; ++k) E[k] = S[k];
      E[38] = S[12];
      E[39] = S[13];
      for (int k = 0; k < 6; ++k) E[12 + k] = S[14 + k];
      E[40] = S[20];
      E[41] = S[21];
    }
  }
  if (infeas_due(p, st)) {
    double T[20];
#pragma unroll
    for (int k = 0; k < 20; ++k) T[k] = 0.0;
    for (int i = threadIdx.x; i < p.K.nred; i += kDecideBlock) {
#pragma unroll
      for (int k = 0; k < 8; ++k) T[k] += p.partE3[8 * i + k];
    }
    for (int i = threadIdx.x; i < p.KT.nred; i += kDecideBlock) {
#pragma unroll
      for (int k = 0; k < 12; ++k) T[8 + k] += p.partE4[12 * i + k];
    }
    block_sum<20, kDecideBlock / 64>(T, red);
    if (threadIdx.x == 0)
      for (int k = 0; k < 20; ++k) E[18 + k] = T[k];
  }
  if (threadIdx.x == 0) eval_decision(st, p, p.tr, E, p.qnorm0, p.cnorm0);
}

// Normalized duality gap (restart metric 1): one pass of the multiplier
// search over the columns (blocks [0, gn)) and the rows (blocks [gn, ...)),
// both candidates, kGapPoints multiplier values each; one partial of kGapAcc
// sums per workgroup.
__global__ __launch_bounds__(kBlock) void k_gap_pass(Params p, int gn) {
  __shared__ double red[kGapAcc * (kBlock / 64)];
  const DevState* st = p.st;
  if (!st->gap_active) return;
  const GapScale g0(st->gap_lam[0], st->omega), g1(st->gap_lam[1], st->omega);
  double acc[kGapAcc];
#pragma unroll
  for (int k = 0; k < kGapAcc; ++k) acc[k] = 0.0;
  const int cur = st->cur;
  if ((int)blockIdx.x < gn) {
    const double* __restrict__ x = sel(cur, p.x[0], p.x[1]);
    for (int j = p.col_base + blockIdx.x * kBlock + threadIdx.x; j < p.col_base + p.n; j += gn * kBlock) {
      gap_col<0>(p, x, g0, j, acc);
      gap_col<1>(p, x, g1, j, acc + 2 * kGapPoints);
    }
  } else {
    const int gm = gridDim.x - gn;
    const double* __restrict__ y = sel(cur, p.y[0], p.y[1]);
    for (int i = p.row_base + (blockIdx.x - gn) * kBlock + threadIdx.x; i < p.row_base + p.m; i += gm * kBlock) {
      gap_row<0>(p, y, g0, i, acc);
      gap_row<1>(p, y, g1, i, acc + 2 * kGapPoints);
    }
  }
  block_sum<kGapAcc>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kGapAcc; ++k) p.partG[kGapAcc * blockIdx.x + k] = acc[k];
  }
}

// Single workgroup: the pass's partials in a fixed order, then gap_step.
__global__ __launch_bounds__(kDecideBlock) void k_gap_step(Params p, int nparts) {
  __shared__ double red[kGapAcc * (kDecideBlock / 64)];
  DevState* st = p.st;
  if (!st->gap_active) return;
  double R[kGapAcc];
#pragma unroll
  for (int k = 0; k < kGapAcc; ++k) R[k] = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kDecideBlock) {
#pragma unroll
    for (int k = 0; k < kGapAcc; ++k) R[k] += p.partG[kGapAcc * i + k];
  }
  block_sum<kGapAcc, kDecideBlock / 64>(R, red);
  if (threadIdx.x == 0) gap_step(st, p, p.tr, R);
}

// x-space part of a restart: z^{n+1,0} = candidate, sums cleared.  The flag
// is cleared by the next k_decide.
__global__ __launch_bounds__(kBlock) void k_restart_x(Params p) {
  const DevState* st = p.st;
  if (!st->restart_flag) return;
  const int cur = st->cur, cand = st->cand_avg;
  double* __restrict__ x = sel(cur, p.x[0], p.x[1]);
  for (int j = p.col_base + blockIdx.x * kBlock + threadIdx.x; j < p.col_base + p.n; j += gridDim.x * kBlock) {
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
  for (int j = p.col_base + blockIdx.x * kBlock + threadIdx.x; j < p.col_base + p.n; j += gridDim.x * kBlock) {
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
  for (int i = p.row_base + blockIdx.x * kBlock + threadIdx.x; i < p.row_base + p.m; i += gridDim.x * kBlock) {
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
  double f = 1.0;
  if (st->status == 5) {   // the unit dual ray of a primal-infeasibility certificate
    y = p.yr[st->ray_src];
    f = st->ray_scale;
  }
  for (int i = p.row_base + blockIdx.x * kBlock + threadIdx.x; i < p.row_base + p.m; i += gridDim.x * kBlock) {
    const double v = p.D1[i] * y[i] * f;
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

// ---------------------------------------------------------------------------- launchers

// Kernel timing (pdlp_profile_attempts): while set, the first kernel of a
// step pass records t0 at its own start and the last records t1 at its own
// end (hipExtLaunchKernelGGL: the runtime takes both at the kernel's
// boundaries, so the interval holds the pass's kernels and the gaps between
// them, not the event packets around them).
static thread_local hipEvent_t g_t0 = nullptr, g_t1 = nullptr;

void set_pass_events(hipEvent_t t0, hipEvent_t t1) {
  g_t0 = t0;
  g_t1 = t1;
}

template <typename F>
static void go(F kernel, dim3 grid, dim3 block, hipStream_t s, const Params& p, bool first, bool last) {
  hipEvent_t a = first ? g_t0 : nullptr, b = last ? g_t1 : nullptr;
  if (a || b) hipExtLaunchKernelGGL(kernel, grid, block, 0, s, a, b, 0, p);
  else hipLaunchKernelGGL(kernel, grid, block, 0, s, p);
}

static inline int elem_grid(int n) {
  int g = (n + kBlock - 1) / kBlock;
  if (g > kElemBlocks) g = kElemBlocks;
  return g < 1 ? 1 : g;
}

// A pass in the SELL-64 layout (sel.cfg selects the workgroup size and
// whether the leading gathered entries are staged in LDS).
template <class Op, typename VT>
static void launch_sell(const Params& p, const DevCsr& M, hipStream_t s) {
  const SellCsr& S = M.sel;
  if (S.cfg == 0) go(k_sell<Op, VT, 1024, true>, dim3(S.grid), dim3(1024), s, p, true, true);
  else if (S.cfg == 1) go(k_sell<Op, VT, 512, true>, dim3(S.grid), dim3(512), s, p, true, true);
  else go(k_sell<Op, VT, 256, false>, dim3(S.grid), dim3(256), s, p, true, true);
}

// One pass of `Op` over its matrix in the matrix's layout, with the
// kernels built for the tiling of M's blocks.
template <class Op, typename VT, int TILE = kTile>
static void launch_op(const Params& p, const DevCsr& M, hipStream_t s) {
  if (M.layout == 4) {
    launch_sell<Op, VT>(p, M, s);
  } else if (M.layout == 0) {
    const int g = M.grid > 0 && M.grid < M.nblocks ? M.grid : M.nblocks;
    go(k_fused<Op, VT, TILE>, dim3(g), dim3(kBlock), s, p, true, true);
  } else {
    const int g = M.grid > 0 && M.grid < M.pan.nsblocks ? M.grid : M.pan.nsblocks;
    go(k_seg<Op, VT, TILE>, dim3(g), dim3(kBlock), s, p, true, false);
    go(k_rows<Op>, dim3(M.rows_grid), dim3(kBlock), s, p, false, true);
  }
}

// A step pass in the LDS-staged layout: the long rows' staged panels and
// then, in the same workgroups, the short rows' column panels (stg.cfg
// selects the workgroup size); then the row pass.
template <class Op, typename VT>
static void launch_staged(const Params& p, const DevCsr& M, hipStream_t s) {
  const StagedCsr& S = M.stg;
  // the grid: every work item, a multiple of 8 (XCD affinity of the short
  // rows' panel blocks)
  const int g = S.sgrid;
  if (S.cfg == 2) go(k_stage<Op, VT, 1024>, dim3(g), dim3(1024), s, p, true, false);
  else if (S.cfg == 1) go(k_stage<Op, VT, 512>, dim3(g), dim3(512), s, p, true, false);
  else go(k_stage<Op, VT, 256>, dim3(g), dim3(256), s, p, true, false);
  go(k_stage_rows<Op, VT>, dim3(S.nlong_groups + S.nrblocks), dim3(kBlock), s, p, false, true);
}

// A step pass over a step view: the view replaces the matrix in the kernels'
// parameters, and its tiling picks the kernels.
template <class Op, int WHICH>
static void launch_view(const Params& p, hipStream_t s) {
  Params q = p;
  DevCsr& M = WHICH ? q.KT : q.K;
  M = WHICH ? p.KTs : p.Ks;
  if (M.layout == 3) {
    if (q.use_f32) launch_staged<Op, float>(q, M, s);
    else launch_staged<Op, double>(q, M, s);
  } else if (M.layout == 4) {
    if (q.use_f32) launch_sell<Op, float>(q, M, s);
    else launch_sell<Op, double>(q, M, s);
  } else if (M.tile == kTileWide) {
    if (q.use_f32) launch_op<Op, float, kTileWide>(q, M, s);
    else launch_op<Op, double, kTileWide>(q, M, s);
  } else {
    if (q.use_f32) launch_op<Op, float>(q, M, s);
    else launch_op<Op, double>(q, M, s);
  }
}

void launch_primal(const Params& p, hipStream_t s) { launch_view<PrimalOp, 1>(p, s); }

void launch_dual(const Params& p, hipStream_t s) { launch_view<DualOp, 0>(p, s); }

void launch_decide(const Params& p, hipStream_t s) {
  hipLaunchKernelGGL(k_decide, dim3(1), dim3(kDecideBlock), 0, s, p);
}

void launch_eval(const Params& p, hipStream_t s) {
  const int ge = elem_grid(p.n);
  hipLaunchKernelGGL(k_eval_x, dim3(ge), dim3(kBlock), 0, s, p);
  // the rows of K~: on an LDS-staged step view of the FP64 matrix, K~x_bar
  // and then K~x with the epilogue, a staged pass each (together 0.6 of the
  // time of one pass gathering both vectors over the evaluation view's column
  // panels, on a skewed LP of 2e7 nonzeros); otherwise that one pass.  The
  // partials come one per workgroup of the pass that ran.
  int n_e1 = p.K.nred;
  if (p.kxb && p.Ks.layout == 3 && !p.use_f32) {
    Params q = p;
    q.K = p.Ks;
    launch_staged<EvalKxbOp, double>(q, q.K, s);
    launch_staged<EvalRowsKxbOp, double>(q, q.K, s);
    n_e1 = p.Ks.nred;
  } else {
    launch_op<EvalRowsOp, double>(p, p.K, s);
  }
  launch_op<EvalColsOp, double>(p, p.KT, s);
  if (p.infeas) {
    launch_op<InfeasRowsOp, double>(p, p.K, s);
    launch_op<InfeasColsOp, double>(p, p.KT, s);
  }
  hipLaunchKernelGGL(k_eval_decide, dim3(1), dim3(kDecideBlock), 0, s, p, ge, n_e1);
  if (p.gap) {
    const int gn = elem_grid(p.n), gm = elem_grid(p.m);
    for (int ph = 0; ph < kGapPasses + 2; ++ph) {
      hipLaunchKernelGGL(k_gap_pass, dim3(gn + gm), dim3(kBlock), 0, s, p, gn);
      hipLaunchKernelGGL(k_gap_step, dim3(1), dim3(kDecideBlock), 0, s, p, gn + gm);
    }
  }
  hipLaunchKernelGGL(k_restart_x, dim3(ge), dim3(kBlock), 0, s, p);
  // K~x of the restart point: one gathered vector, like the dual step, so it
  // takes the dual step's view (and its matrix precision)
  launch_view<RestartYOp, 0>(p, s);
}

void launch_init(const Params& p, const double* xs, const double* ys, hipStream_t s) {
  hipLaunchKernelGGL(k_init_x, dim3(elem_grid(p.n)), dim3(kBlock), 0, s, p, xs);
  hipLaunchKernelGGL(k_init_y, dim3(elem_grid(p.m)), dim3(kBlock), 0, s, p, ys);
}

void launch_output(const Params& p, hipStream_t s) {
  launch_op<OutputOp, double>(p, p.KT, s);
  hipLaunchKernelGGL(k_output_y, dim3(elem_grid(p.m)), dim3(kBlock), 0, s, p);
}

void launch_set_limit(DevState* st, int status, hipStream_t s) {
  hipLaunchKernelGGL(k_set_limit, dim3(1), dim3(1), 0, s, st, status);
}

}  // namespace pdlp
