// Internal layout shared by the host runtime and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "pdlp.h"

namespace pdlp {

constexpr int kBlock = 256;        // threads per workgroup (4 wavefronts of 64)
constexpr int kTile = 3072;        // nonzeros staged in LDS per row block (12 per thread)
constexpr int kTileWide = 6144;    // the wider tiling a step pass may take (24 per thread)
constexpr int kMaxRows = 1024;     // rows per row block
constexpr int kElemBlocks = 2048;  // fixed grid of the row-wise kernels (deterministic partials)
constexpr int kPanels = 8;         // column panels of the split layout = XCDs of the chip
// normalized duality gap: multiplier values per pass, multisection passes, and
// the sums a pass reduces (per candidate: ||d||^2 and g'd at each value)
constexpr int kGapPoints = 4;
constexpr int kGapPasses = 22;
constexpr int kGapAcc = 2 * 2 * kGapPoints;

// A row block of a CSR matrix: rows [r0, r1).  Either short rows with at most
// kTile nonzeros in total (handled in one pass through LDS), or one long row
// with more than kTile nonzeros (swept by the whole workgroup).
struct RowBlock {
  int32_t r0, r1;
};

// Column-panel ("split") layout of a CSR matrix.  The columns are cut into
// kPanels ranges of about equal nonzero count; the nonzeros of row r that fall
// in panel p form segment (r, p).  Segments are stored panel-major (all of
// panel 0, then panel 1, ...), rows ascending inside a panel; the phase-1
// blocks are interleaved so that workgroup i only touches panel i % kPanels.
// Workgroups are dispatched round-robin over the 8 XCDs, so each XCD gathers
// from one eighth of the vector, which then stays in its own L2.
struct PanelCsr {
  int32_t nseg;
  int32_t nsblocks;
  const int32_t* seg_ptr;   // [nseg+1] start of each segment in pci / pv (panel-major)
  const int32_t* slot_seg;  // [nseg]   segment of each row-major slot
  const int32_t* row_seg;   // [nrows+1] row r's slots are [row_seg[r], row_seg[r+1]), in panel order
  const int32_t* pci;       // [nnz] column indices in segment order
  const double* pv;         // [nnz] FP64 values in segment order
  const float* pvf;         // [nnz] FP32 values in segment order (nullptr unless FP32 steps)
  const RowBlock* sblocks;  // [nsblocks] phase-1 blocks (rows of the segment "matrix")
  double* part;             // [2 * nseg] segment sums in segment (panel-major) order, so that each
                            // workgroup's stores are contiguous and stay on its own XCD
};

// LDS-staged panel layout of a CSR matrix for a step pass (one gathered
// vector).  The long rows (at least 256 nonzeros; the descending-length row
// order numbers them first) are cut by columns into panels of kStageWidth
// columns; the nonzeros of long row r in panel p form segment (r, p).  Inside
// a panel the segments are sorted by length (longest first) and grouped in
// chunks of kStageLanes, one segment per lane of a wavefront, stored
// lane-interleaved (entry k of lane l at coff + 64 k + l) with zeros padding
// each lane up to the chunk's longest segment, column indices relative to the
// panel (16 bits).  Phase 1 (k_stage): a work item (one workgroup) is a run of one
// panel's chunks; it copies the panel's slice of the gathered vector into LDS
// once, then each wavefront sums whole chunks (coalesced loads, every gather
// an LDS read, no barrier) and stores one sum per segment, at [panel][row]
// of a dense array (a panel's items run on one XCD, whose L2 merges those
// stores).  The short rows take column panels of their own, one per XCD (the
// step view's PanelCsr), summed by the same workgroups after their items:
// each XCD then gathers from one eighth of the vector, which stays in its L2,
// where random gathers from the whole vector would pull a cache line from
// memory for nearly every nonzero; rows of one nonzero (their gathers run in
// address order) are left out.  Phase 2 (k_stage_rows): a thread per short
// row adds its panel sums in panel order (or takes its one product); 64 long
// rows per workgroup add their dense segment sums (consecutive lanes read
// consecutive entries); every row runs the epilogue.
constexpr int kStageWidth = 16384;   // columns per panel: 128 KB of FP64 in LDS (at most 65536: 16-bit indices)
constexpr int kStageLanes = 64;      // segments per chunk
struct StagedCsr {
  int32_t nwork;            // phase-1 work items
  int32_t ncols;
  int32_t nseg;             // segments of the long rows
  int32_t cfg;              // phase-1 workgroup size: 0: 256, 1: 512, 2: 1024 threads
  int32_t rlong;            // rows [0, rlong) are the long rows
  int32_t nlong_groups;     // phase-2 workgroups of the long rows
  int32_t nrblocks;         // phase-2 workgroups of the short rows (one row per thread)
  int32_t sgrid;            // k_stage's workgroups (every work item, a multiple of 8)
  const int32_t* wpanel;    // [nwork] panel of each work item
  const int32_t* wchunk;    // [2 nwork] chunk range [wchunk[2w], wchunk[2w+1]) of work item w (empty: a pad)
  const int32_t* coff;      // [nchunk] first entry of each chunk
  const int32_t* clen;      // [nchunk] entries per lane (the chunk's longest segment)
  const int32_t* cseg;      // [nchunk+1] first segment of each chunk
  const uint16_t* pci;      // column index relative to the panel (0 on padding)
  const double* pv;         // FP64 values (0 on padding)
  const float* pvf;         // FP32 values (nullptr unless FP32 steps)
  int32_t npan;             // panels
  int32_t pad2;
  const int32_t* srow;      // [nseg] the long row of each segment
  double* part;             // [npan * rlong] segment sums, panel-major and by row inside a panel
                            // (zero where a row has no nonzero in a panel: never written)
};

// SELL-64 layout of a step view (layout 4): the rows are cut into chunks of
// 64 consecutive rows, stored lane-interleaved (entry k of the chunk's row l
// at coff + 64 k + l) and zero-padded to the chunk's longest row.  With the
// rows numbered by descending length (columns renumbered for K~', rows for
// K~) a chunk's rows have nearly equal lengths, so the padding is small.  A
// wavefront sums a chunk, one row per lane, with coalesced loads and no
// cross-lane reduction; each workgroup first copies the leading `hot` entries
// of the gathered vector into LDS (the rows of the other matrix numbered
// first are the longest, so their entries are gathered most often) and reads
// them there.
constexpr int kSellHot = 8192;   // leading gathered entries staged in LDS: 64 KB of FP64
struct SellCsr {
  int32_t nchunks;
  int32_t hot;              // entries of the gathered vector staged in LDS (cfg 0, 1): min(kSellHot, its length)
  int32_t cfg;              // 0: 1024-thread workgroups with the LDS slice; 1: 512 threads with it;
                            // 2: 256 threads without it
  int32_t grid;             // workgroups of the persistent launch (one reduction partial each)
  const int32_t* coff;      // [nchunks] first entry of each chunk
  const int32_t* clen;      // [nchunks] entries per lane (the chunk's longest row)
  const int32_t* sci;       // column indices (0 on padding)
  const double* sv;         // FP64 values (0 on padding)
  const float* svf;         // FP32 values (nullptr unless FP32 steps)
};

struct DevCsr {
  const int32_t* rp;
  const int32_t* ci;
  const double* v;        // FP64 scaled values
  const float* vf;        // FP32-rounded scaled values (nullptr unless FP32 steps)
  const RowBlock* blocks; // long rows first, then runs of short rows
  int32_t nblocks;
  int32_t nrows;
  int32_t layout;         // 0: fused row blocks; 1: column panels (two phases); 3: LDS-staged panels (stg);
                          // 4: SELL-64 chunks (sel)
  int32_t remap;          // fused layout: contiguous block ranges per XCD
  int32_t nred;           // reduction partials of a pass over this matrix
  int32_t rows_grid;      // grid of the phase-2 (row-wise) kernels
  int32_t grid;           // grid of the row-block (phase-1) kernels: 0 = one workgroup per block,
                          // else a persistent grid (a multiple of 8) looping over the blocks
  PanelCsr pan;
  int32_t tile;           // nonzeros per block of `blocks` and `pan.sblocks`: 0 = kTile, or kTileWide
  StagedCsr stg;          // layout 3 (step views only): LDS-staged panels of the long rows
  SellCsr sel;            // layout 4 (step views only): SELL-64 chunks
};

// Solver state in device memory.  The first 16 bytes are the status word the
// host polls.
struct DevState {
  int32_t done;           // 1 once a status is set
  int32_t status;         // PDLP_OPTIMAL ... (0 while running)
  int64_t k;              // accepted steps
  // step state
  double eta;             // step size of the next attempt
  double eta_hat;
  double omega;
  double sum_eta;         // sum of accepted step sizes in the epoch
  double pending_w;       // step size of the accepted iterate not yet added to the sums
  double kkt0, kkt_prev;
  int64_t t;              // accepted steps in the epoch
  int64_t attempts, restarts, evals, k_last_eval;
  int32_t cur;            // buffer index of the current iterate
  int32_t has_pending;
  int32_t need_eval;      // an evaluation is due (P accepted steps since the last one)
  int32_t initial;        // the evaluation of the starting point
  int32_t restart_flag;   // the evaluation asked for a restart (applied by the restart kernels)
  int32_t cand_avg;       // restart candidate / returned point is the average
  int32_t ret_avg;
  int32_t ray_src;        // infeasibility certificate: 0 the last accepted step, 1 the epoch displacement
  // termination parameters of this solve
  double eps_rel;
  int64_t max_iter;
  // last evaluation, returned point
  double rel_kkt, rel_gap, rel_p, rel_d, pobj, dobj;
  // infeasibility certificate (statuses 5, 6): 1 / ||ray|| and the unit ray's objective and residual
  double ray_scale, ray_obj, ray_res;
  // normalized duality gap (restart metric 1): per candidate (current, average)
  // the multiplier search of the trust-region problem, run between evaluation
  // and restart while gap_active
  double gap_lam[2][4];   // the multiplier values of the next pass
  double gap_lo[2], gap_hi[2], gap_r[2], gap_rho[2];
  double gap_dx2[2], gap_dy2[2];   // ||x_c - x0||^2, ||y_c - y0||^2 for the primal weight update
  int32_t gap_mode[2];    // 0 searching, 1 ball not binding (multiplier lo), 2 rho = 0
  int32_t gap_phase, gap_active;
  int64_t n_att, n_eval;  // trace entries written
};

struct Trace {
  int64_t cap;
  int64_t* att_k; double* att_eta; double* att_etabar; int8_t* att_acc;
  int64_t* ev_k; double* ev_kkt_cur; double* ev_kkt_avg; int8_t* ev_cand; int8_t* ev_reason;
  double* ev_omega;
};

struct Params {
  DevCsr K;     // m rows
  DevCsr KT;    // n rows
  // the views the step passes take of K and K': the
  // same arrays, with a row-block tiling of their own (kTile or kTileWide)
  DevCsr Ks, KTs;
  int32_t m, n;
  int32_t use_f32;
  int32_t pad0;
  // first row / column of the elementwise passes (0; an LP of a batch continued
  // on these kernels works on its slice of the packed vectors)
  int32_t row_base, col_base;
  // iterates (double-buffered where a step writes a new one)
  double* x[2];
  double* y[2];
  double* kx[2];          // K~ x for the current x (attempt precision)
  double* dx;             // x' - x of the current attempt
  double* xsum; double* ysum;
  double* xbar; double* ybar;
  double* x0; double* y0;
  // problem (scaled, >= form)
  const double* c; const double* q; const double* l; const double* u;
  const int8_t* ineq;
  const int8_t* le;
  const double* D1; const double* D2;
  // outputs of the last solve (user orientation)
  double* xo; double* yo; double* rco;
  // one partial (NV doubles) per workgroup, added in order by the decision kernels
  double* partA;          // ||dx||^2
  double* partB;          // ||dy||^2, dy'K~dx
  double* partE0;         // [kElemBlocks * 4]
  double* partE1;         // 8 per partial
  double* partE2;         // 6 per partial
  DevState* st;
  Trace tr;
  // constants
  int64_t P;
  double beta_suff, beta_nec, beta_art, theta, eps_zero;
  double tie_rel;         // relative band in which the candidate comparison is a tie
  int32_t omega_power;
  double qnorm0, cnorm0;
  // infeasibility detection: candidate rays of the last evaluation (scaled
  // space, projected), their partials, the tolerance (infeas = 0: off)
  int32_t infeas;
  int32_t infeas_every;   // evaluations per certificate test
  double eps_infeas;
  double* xr[2];          // [n] each: the last step's and the epoch displacement's x, projected
  double* yr[2];          // [m] each: the same for y, clipped at 0 on inequality rows
  double* partE3;         // 8 per partial of the rows of K~
  double* partE4;         // 12 per partial of the rows of K~'
  // normalized duality gap (gap = 1): K~x, K~x_bar and K~'y, K~'y_bar of the
  // evaluation, and 16 partials per elementwise block of the multiplier passes
  int32_t gap;
  double* kxe[2];
  double* ktye[2];
  double* partG;
  // [m]: K~x_bar of an evaluation whose rows of K~ run as two one-vector
  // passes on the LDS-staged step view (FP64 matrix); null otherwise
  double* kxb;
};

constexpr int32_t kPaused = 16;  // internal status of a batched LP handed to the single-LP kernels

// Batched solve (many independent LPs packed block-diagonally into one Params).
struct BatchParams {
  int32_t count;            // LPs in the queue
  int32_t trace_lp;         // LP whose decisions are traced (-1: none)
  const int32_t* order;     // [count] queue order (LP indices)
  const int32_t* row_off;   // [nlp+1]
  const int32_t* col_off;   // [nlp+1]
  const uint8_t* lanes;     // [2*nlp] K~ rows, K~' rows: 0 = LDS-tiled row blocks, else lanes per row
  const RowBlock* bk;       // row blocks of every LP's rows of K~ (LP b: [bk_off[b], bk_off[b+1]))
  const int32_t* bk_off;
  const RowBlock* bt;       // row blocks of every LP's rows of K~'
  const int32_t* bt_off;
  DevState* st;             // [nlp]
  const double* norms;      // [4*nlp] squared norms: ||q||, ||c|| (unscaled), ||c~||, ||q~|| (scaled)
  const double* kmax;       // [nlp] max |K~_ij|
  const double* omega_warm; // [nlp] warm-start primal weight (<= 0: default)
  const int8_t* warm;       // [nlp] 1: start from the warm-start slices of wx / wy
  const double* wx;
  const double* wy;
  uint32_t* queue;          // next queue slot (zero before the launch)
  const uint64_t* t0;       // wall-clock stamp taken just before the launch
  uint64_t ticks;           // time limit in wall-clock ticks (0: none)
  int64_t max_reject;       // consecutive rejected attempts that count as a numerical failure
  int64_t pause_at;         // accepted steps after which an LP stops at its next evaluation with
                            // status kPaused (0: never)
  int32_t resume;           // 1: the queued LPs were paused; continue each from its state in st
  int32_t pad1;
  int32_t lds_m, lds_n;     // LDS room for an LP's y, dx and row pointers (0, 0: all from global memory)
  int32_t lds_bk, lds_bt;   // LDS room for an LP's block descriptors of K~, K~'
  double eps_rel;
  int64_t max_iter;
  double eps_zero;
};

// One LP, or LPs packed block-diagonally, on the host (user orientation).
struct HostLP {
  int32_t m = 0, n = 0;
  int64_t nnz = 0;
  std::vector<int32_t> rp, ci;
  std::vector<double> v, c, b, l, u;
  std::vector<int8_t> rt;
};

// Validate `count` LPs (host or device arrays) and pack them block-diagonally;
// returns PDLP_OK or an error code with the reason (naming the first bad LP).
int pack_problems(const pdlp_problem* ps, int32_t count, void* hip_stream, HostLP& H, std::vector<int32_t>& row_off,
                  std::vector<int32_t>& col_off, std::vector<int64_t>& nnz_b, std::string& why);

// Presolve-lite record (presolve.cpp): what was removed and how to undo it.
struct Presolve {
  int status = 0;                      // 0, or PDLP_PRIMAL_INFEASIBLE / PDLP_DUAL_INFEASIBLE found by presolve
  std::vector<uint8_t> row_on, col_on; // kept rows / columns
  std::vector<int32_t> rows, cols;     // their indices, ascending
  std::vector<double> xfix;            // values of the removed columns
  std::vector<double> lo, hi;          // final bounds
  std::vector<int32_t> lo_row, hi_row; // singleton row that set each bound (-1: the column's own)
  std::vector<int32_t> order;          // removed columns in removal order
  double offset = 0.0;                 // objective of the removed columns
  std::vector<double> b;               // right-hand sides after the reductions (kept rows)
  std::vector<int32_t> cp, cr;         // the original matrix by columns
  std::vector<double> cv;
};

int presolve_lp(const HostLP& H, HostLP& R, Presolve& P);
void postsolve_lp(const HostLP& H, const Presolve& P, const double* xr, const double* yr, const double* lamr,
                  double* x, double* y, double* lam, bool ray);

hipError_t setup_transpose(int m, int n, int64_t nnz, const int32_t* ci, const double* v, const int32_t* rowid,
                           int32_t* rpT, int32_t* ciT, double* vT, int32_t* rowidT, int32_t* perm_out,
                           hipStream_t s);

}  // namespace pdlp
