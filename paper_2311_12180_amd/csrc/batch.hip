// Batched restarted PDHG: many independent LPs in one persistent launch (see
// the comment of the batched-LP section below).  Uses the shared ops and
// decision functions of pdlp_ops.h, so every LP runs the same arithmetic as
// the single-LP kernels.
#include <math.h>

#include "pdlp_ops.h"

namespace pdlp {

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

constexpr int kBB = 512;    // threads of a batch workgroup (8 wavefronts): one LP at a time
constexpr int kBT = 4096;   // nonzeros per LDS tile of the batched sweeps (8 per thread)
constexpr int kBW = kBB / 64;

// Row pointers of an LP from an LDS copy (global row index r).
struct LdsRowPtr {
  const int* p;
  int base;
  __device__ int operator[](int r) const { return p[r - base]; }
};

// Gather from an LDS copy of an LP's slice of a vector (global index i).
struct LdsGather {
  const double* v;
  int base;
  __device__ void operator()(int i, double* g) const { g[0] = v[i - base]; }
};
template <class Op>
struct OpGather {
  const Op& op;
  __device__ void operator()(int i, double* g) const { op.gather(i, g); }
};

// Row sweep of one LP's rows [rb, re) with L lanes per row; epi runs on the
// group's first lane.
template <int NV, typename VT, class RP, class G, class E>
__device__ __forceinline__ void lane_rows(const RP& rp, const int32_t* __restrict__ ci, const VT* __restrict__ v,
                                          int rb, int re, int L, const G& gather, const E& epi) {
  const int groups = kBB / L;
  const int grp = threadIdx.x / L, lane = threadIdx.x - grp * L;
  for (int r = rb + grp; r < re; r += groups) {
    double s[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k] = 0.0;
    const int e1 = rp[r + 1];
    for (int e = rp[r] + lane; e < e1; e += L) {
      const double a = (double)v[e];
      double g[NV];
      gather(ci[e], g);
#pragma unroll
      for (int k = 0; k < NV; ++k) s[k] += a * g[k];
    }
    for (int off = L >> 1; off > 0; off >>= 1) {
#pragma unroll
      for (int k = 0; k < NV; ++k) s[k] += __shfl_down(s[k], off, L);
    }
    if (lane == 0) epi(r, s);
  }
}

// One pass over an LP's rows: its LDS-tiled row blocks [b0, b1) when L = 0
// (the single-LP sweep at batch width), else rows [rb, re) with L lanes per
// row.  Ends with a workgroup barrier.
// An LP's view of one matrix: its rows [rb, re), its row blocks, and where
// its row pointers and block descriptors are read from (LDS copies when the
// LP fits, else global memory).
struct LpMat {
  const int32_t* grp;       // global row pointers
  const int* lrp;           // LDS copy of rp[rb .. re] (nullptr: use grp)
  const RowBlock* blocks;   // block descriptors (LDS copy or global), blocks [0, nb)
  int nb, rb, re;
};

template <int NV, typename VT, class RP, class G, class E>
__device__ __forceinline__ void sweep_rp(const RP& rp, const LpMat& L_, const int32_t* __restrict__ ci,
                                         const VT* __restrict__ v, int L, const G& gather, const E& epi, double* lds,
                                         double* red) {
  if (L == 0) {
    for (int j = 0; j < L_.nb; ++j) {
      // two gathered vectors (the evaluations): load each tile in two halves
      spmv_block<NV, VT, kBB, kBT, NV>(rp, ci, v, L_.blocks[j], lds, red, gather, epi);
      __syncthreads();
    }
  } else {
    lane_rows<NV, VT>(rp, ci, v, L_.rb, L_.re, L, gather, epi);
    __syncthreads();
  }
}

// One pass over an LP's rows: its LDS-tiled row blocks when L = 0 (the
// single-LP sweep at batch width), else its rows with L lanes per row.  Ends
// with a workgroup barrier.
template <bool LV, int NV, typename VT, class G, class E>
__device__ __forceinline__ void sweep(const LpMat& M, const int32_t* __restrict__ ci, const VT* __restrict__ v, int L,
                                      const G& gather, const E& epi, double* lds, double* red) {
  if constexpr (LV) sweep_rp<NV, VT>(LdsRowPtr{M.lrp, M.rb}, M, ci, v, L, gather, epi, lds, red);
  else sweep_rp<NV, VT>(M.grp, M, ci, v, L, gather, epi, lds, red);
}

// Steps of one attempt with the gathered vector taken from global memory
// (the op's own gather) or from the LP's LDS copy.
template <bool LV, typename VT, class Op>
__device__ __forceinline__ void step_sweep(const LpMat& M, const int32_t* ci, const VT* v, int L, const Op& op,
                                           double* acc, const double* lvec, int lbase, double* lds, double* red) {
  const auto epi = [&](int r, const double* s) { op.epi(r, s, acc); };
  if constexpr (LV) sweep<LV, 1, VT>(M, ci, v, L, LdsGather{lvec, lbase}, epi, lds, red);
  else sweep<LV, 1, VT>(M, ci, v, L, OpGather<Op>{op}, epi, lds, red);
}

template <bool LV, int NV, class Op>
__device__ __forceinline__ void plain_sweep(const LpMat& M, const DevCsr& D, int L, const Op& op, double* acc,
                                            double* lds, double* red) {
  sweep<LV, NV, double>(M, D.ci, D.v, L, OpGather<Op>{op}, [&](int r, const double* s) { op.epi(r, s, acc); },
                        lds, red);
}

// One candidate's sums of a normalized-duality-gap pass over an LP's columns
// and rows, reduced into out[0 .. 2 kGapPoints).
template <int C>
__device__ __forceinline__ void gap_sweep(const Params& p, const DevState* S, int c0, int c1, int r0, int r1,
                                       double* red, double* out) {
  const GapScale g(S->gap_lam[C], S->omega);
  double acc[2 * kGapPoints];
#pragma unroll
  for (int k = 0; k < 2 * kGapPoints; ++k) acc[k] = 0.0;
  const int cur = S->cur;
  const double* __restrict__ x = sel(cur, p.x[0], p.x[1]);
  const double* __restrict__ y = sel(cur, p.y[0], p.y[1]);
  for (int j = c0 + threadIdx.x; j < c1; j += kBB) gap_col<C>(p, x, g, j, acc);
  for (int i = r0 + threadIdx.x; i < r1; i += kBB) gap_row<C>(p, y, g, i, acc);
  block_sum<2 * kGapPoints, kBW>(acc, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 2 * kGapPoints; ++k) out[k] = acc[k];
  __syncthreads();
}

template <bool LV>
__device__ void batch_solve_one(const Params& p, const BatchParams& bp, int b, DevState* S, double* red,
                                double* E, double* lds, double* ly, double* ldx, int* lrk, int* lrt, RowBlock* lbk,
                                RowBlock* lbt) {
  const int r0 = bp.row_off[b], r1 = bp.row_off[b + 1];
  const int c0 = bp.col_off[b], c1 = bp.col_off[b + 1];
  const int LK = bp.lanes[2 * b], LT = bp.lanes[2 * b + 1];
  const int k0 = bp.bk_off[b], k1 = bp.bk_off[b + 1], t0 = bp.bt_off[b], t1 = bp.bt_off[b + 1];
  const Trace tr = b == bp.trace_lp ? p.tr : Trace{};
  const double qn0 = sqrt(bp.norms[4 * b]), cn0 = sqrt(bp.norms[4 * b + 1]);
  const bool f32 = p.use_f32 != 0;
  // LDS copies of the gathered step vectors, row pointers and block
  // descriptors when the LP fits (else everything is read from global memory)
  // (LV: the launch sized the LDS for the batch's largest LP, so every LP fits)
  constexpr bool lv = LV;
  if (lv) {
    for (int i = threadIdx.x; i <= r1 - r0; i += kBB) lrk[i] = p.K.rp[r0 + i];
    for (int j = threadIdx.x; j <= c1 - c0; j += kBB) lrt[j] = p.KT.rp[c0 + j];
    for (int q = threadIdx.x; q < k1 - k0; q += kBB) lbk[q] = bp.bk[k0 + q];
    for (int q = threadIdx.x; q < t1 - t0; q += kBB) lbt[q] = bp.bt[t0 + q];
  }
  const LpMat mk{p.K.rp, lv ? lrk : nullptr, lv ? lbk : bp.bk + k0, k1 - k0, r0, r1};
  const LpMat mt{p.KT.rp, lv ? lrt : nullptr, lv ? lbt : bp.bt + t0, t1 - t0, c0, c1};
  if (bp.resume) {
    // a paused LP: its state block and vectors are where the pause left them
    if (threadIdx.x == 0) {
      *S = bp.st[b];
      S->status = 0;
      S->done = 0;
    }
  } else {
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
    for (int j = c0 + threadIdx.x; j < c1; j += kBB) {
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
    for (int i = r0 + threadIdx.x; i < r1; i += kBB) {
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
  }
  __syncthreads();
  int64_t k_seen = 0, rejected = 0;  // thread 0: accepted steps at the last attempt, rejections since
  for (;;) {
    if (S->need_eval) {
      // --- evaluation: averages, eq. (kkt) pieces, Section 4.1 quantities.
      // Each pass is reduced right after it runs (element by element, as one
      // block_sum of all 18 would) to keep few accumulators live.
      {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        const int cur = S->cur, init = S->initial, pend = S->has_pending;
        const double pw = S->pending_w, se = S->sum_eta;
        const double* __restrict__ x = sel(cur, p.x[0], p.x[1]);
        const double* __restrict__ xp = sel(cur, p.x[1], p.x[0]);
        const bool rays = infeas_due(p, S);
        for (int j = c0 + threadIdx.x; j < c1; j += kBB) {
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
        block_sum<4, kBW>(acc, red);
        if (threadIdx.x == 0)
          for (int k = 0; k < 4; ++k) E[k] = acc[k];
      }
      {
        double acc[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) acc[k] = 0.0;
        const EvalRowsOp op(p, S);
        plain_sweep<LV, 2>(mk, p.K, LK, op, acc, lds, red);
        block_sum<10, kBW>(acc, red);
        if (threadIdx.x == 0) {
          for (int k = 0; k < 8; ++k) E[4 + k] = acc[k];
          E[38] = acc[8];
          E[39] = acc[9];
        }
      }
      {
        double acc[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] = 0.0;
        const EvalColsOp op(p, S);
        plain_sweep<LV, 2>(mt, p.KT, LT, op, acc, lds, red);
        block_sum<8, kBW>(acc, red);
        if (threadIdx.x == 0) {
          for (int k = 0; k < 6; ++k) E[12 + k] = acc[k];
          E[40] = acc[6];
          E[41] = acc[7];
        }
      }
      if (infeas_due(p, S)) {
        // Section 2.2 infeasibility certificates (the x-space rays were
        // written above; the rows pass writes the y-space rays)
        __syncthreads();
        {
          double acc[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) acc[k] = 0.0;
          const InfeasRowsOp op(p, S);
          plain_sweep<LV, 2>(mk, p.K, LK, op, acc, lds, red);
          block_sum<8, kBW>(acc, red);
          if (threadIdx.x == 0)
            for (int k = 0; k < 8; ++k) E[18 + k] = acc[k];
        }
        __syncthreads();
        {
          double acc[12];
#pragma unroll
          for (int k = 0; k < 12; ++k) acc[k] = 0.0;
          const InfeasColsOp op(p, S);
          plain_sweep<LV, 2>(mt, p.KT, LT, op, acc, lds, red);
          block_sum<12, kBW>(acc, red);
          if (threadIdx.x == 0)
            for (int k = 0; k < 12; ++k) E[26 + k] = acc[k];
        }
      }
      if (threadIdx.x == 0) eval_decision(S, p, tr, E, qn0, cn0);
      __syncthreads();
      if (S->gap_active) {
        // normalized duality gap: the multiplier search's passes over this LP,
        // then the restart decision (in gap_step after the last pass)
        __syncthreads();   // (the K~x / K~'y products of the evaluation are in global memory)
        // (one candidate at a time, to keep the registers of this loop few;
        // E, no longer needed, collects the pass's sums)
        while (S->gap_active) {
          gap_sweep<0>(p, S, c0, c1, r0, r1, red, E);
          gap_sweep<1>(p, S, c0, c1, r0, r1, red, E + 2 * kGapPoints);
          if (threadIdx.x == 0) gap_step(S, p, tr, E);
          __syncthreads();
        }
      }
      if (S->restart_flag) {
        const int cur = S->cur, cand = S->cand_avg;
        double* __restrict__ x = sel(cur, p.x[0], p.x[1]);
        for (int j = c0 + threadIdx.x; j < c1; j += kBB) {
          const double xc = cand ? p.xbar[j] : x[j];
          x[j] = xc;
          p.x0[j] = xc;
          p.xsum[j] = 0.0;
        }
        __syncthreads();
        const RestartYOp op(p, S);
        double dummy[1];
        const auto epi = [&](int r, const double* s) { op.epi(r, s, dummy); };
        if (f32) sweep<LV, 1, float>(mk, p.K.ci, p.K.vf, LK, OpGather<RestartYOp>{op}, epi, lds, red);
        else sweep<LV, 1, double>(mk, p.K.ci, p.K.v, LK, OpGather<RestartYOp>{op}, epi, lds, red);
        if (threadIdx.x == 0) S->restart_flag = 0;
      }
      // hand a long-running LP to the single-LP kernels at this clean point
      // (right after an evaluation, its state complete in S and global memory)
      if (threadIdx.x == 0 && bp.pause_at > 0 && !S->done && S->k >= bp.pause_at) {
        S->status = kPaused;
        S->done = 1;
      }
    } else {
      // --- one attempt of Algorithm 2
      double acc[3] = {0.0, 0.0, 0.0};
      if (lv) {   // the current y, gathered by the primal sweep
        const double* __restrict__ y = sel(S->cur, p.y[0], p.y[1]);
        for (int i = r0 + threadIdx.x; i < r1; i += kBB) ly[i - r0] = y[i];
        __syncthreads();
      }
      {
        const PrimalOp op(p, S);
        if (f32) step_sweep<LV>(mt, p.KT.ci, p.KT.vf, LT, op, acc, lv ? ly : nullptr, r0, lds, red);
        else step_sweep<LV>(mt, p.KT.ci, p.KT.v, LT, op, acc, lv ? ly : nullptr, r0, lds, red);
      }
      if (lv) {   // dx = x' - x, gathered by the dual sweep
        for (int j = c0 + threadIdx.x; j < c1; j += kBB) ldx[j - c0] = p.dx[j];
        __syncthreads();
      }
      {
        const DualOp op(p, S);
        if (f32) step_sweep<LV>(mk, p.K.ci, p.K.vf, LK, op, acc + 1, lv ? ldx : nullptr, c0, lds, red);
        else step_sweep<LV>(mk, p.K.ci, p.K.v, LK, op, acc + 1, lv ? ldx : nullptr, c0, lds, red);
      }
      block_sum<3, kBW>(acc, red);
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
  // --- output of this LP (as the output op and k_output_y); a paused LP gets
  // its output from the single-LP kernels that finish it
  if (S->status != kPaused) {
    const OutputOp op(p, S);
    double dummy[1];
    plain_sweep<LV, 1>(mt, p.KT, LT, op, dummy, lds, red);
    const int cur = S->cur, ra = S->ret_avg;
    const double* __restrict__ y = ra ? p.ybar : sel(cur, p.y[0], p.y[1]);
    double f = 1.0;
    if (S->status == 5) {   // the unit dual ray of a primal-infeasibility certificate
      y = p.yr[S->ray_src];
      f = S->ray_scale;
    }
    for (int i = r0 + threadIdx.x; i < r1; i += kBB) {
      const double v = p.D1[i] * y[i] * f;
      p.yo[i] = p.le[i] ? -v : v;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) bp.st[b] = *S;
}

// Persistent batch solver: every workgroup takes LPs from the queue until it
// is empty, so the launch ends when every LP has been solved.  Dynamic LDS:
// the tile staging (2 x kBT doubles), then (when bp.lds_m > 0) room for an
// LP's y (lds_m doubles), dx (lds_n doubles), row pointers of K~ and K~'
// (lds_m + 1, lds_n + 1 ints) and block descriptors (lds_bk, lds_bt).
template <bool LV>
__global__ __launch_bounds__(kBB) void k_batch(Params p, BatchParams bp) {
  extern __shared__ double dyn[];
  __shared__ DevState S;
  __shared__ double red[12 * kBW];
  __shared__ double E[42];
  __shared__ int slot;
  double* lds = dyn;
  double* ly = bp.lds_m > 0 ? dyn + 2 * kBT : nullptr;
  double* ldx = ly ? ly + bp.lds_m : nullptr;
  int* lrk = ly ? reinterpret_cast<int*>(ldx + bp.lds_n) : nullptr;
  int* lrt = ly ? lrk + bp.lds_m + 1 : nullptr;
  RowBlock* lbk = ly ? reinterpret_cast<RowBlock*>(lrt + bp.lds_n + 1) : nullptr;
  RowBlock* lbt = ly ? lbk + bp.lds_bk : nullptr;
  for (;;) {
    if (threadIdx.x == 0) slot = (int)atomicAdd(bp.queue, 1u);
    __syncthreads();
    const int q = slot;
    __syncthreads();
    if (q >= bp.count) break;
    batch_solve_one<LV>(p, bp, bp.order[q], &S, red, E, lds, ly, ldx, lrk, lrt, lbk, lbt);
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

size_t batch_lds_bytes(const BatchParams& bp) {
  size_t b = sizeof(double) * 2 * (size_t)kBT;
  if (bp.lds_m > 0)
    b += sizeof(double) * ((size_t)bp.lds_m + bp.lds_n) + sizeof(int) * ((size_t)bp.lds_m + bp.lds_n + 2) +
         sizeof(RowBlock) * ((size_t)bp.lds_bk + bp.lds_bt);
  return b;
}

hipError_t batch_prepare(size_t lds_bytes) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_batch<false>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k_batch<true>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
}

void launch_batch(const Params& p, const BatchParams& bp, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, s, const_cast<uint64_t*>(bp.t0));
  if (bp.lds_m > 0) hipLaunchKernelGGL(k_batch<true>, dim3(grid), dim3(kBB), batch_lds_bytes(bp), s, p, bp);
  else hipLaunchKernelGGL(k_batch<false>, dim3(grid), dim3(kBB), batch_lds_bytes(bp), s, p, bp);
}

int batch_occupancy(size_t lds_bytes) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<true>, kBB, lds_bytes) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

int batch_tile() { return kBT; }

int batch_static_lds() {
  hipFuncAttributes a{};
  if (hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_batch<true>)) != hipSuccess) return 4096;
  return (int)a.sharedSizeBytes;
}

void launch_seg_sumsq(int nlp, const int32_t* off, const double* a, double* out, int stride, int slot, hipStream_t s) {
  hipLaunchKernelGGL(k_seg_sumsq, dim3((nlp + 255) / 256), dim3(256), 0, s, nlp, off, a, out, stride, slot);
}

void launch_seg_absmax(int nlp, const int32_t* row_off, const int32_t* rp, const double* v, double* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_seg_absmax, dim3((nlp + 255) / 256), dim3(256), 0, s, nlp, row_off, rp, v, out);
}


}  // namespace pdlp
