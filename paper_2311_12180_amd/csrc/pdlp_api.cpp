// C ABI and host runtime of the MI355X restarted-PDHG LP solver.
//
// pdlp_create validates the LP on the host, uploads it once, and builds the
// scaled >=-form problem on the device (normalisation, transpose, Section 2.2
// preconditioning).  pdlp_solve runs Algorithm 1 as a captured hipGraph of
// attempt slots (primal kernel, dual kernel, single-workgroup Algorithm 2 decision)
// followed by the evaluation/restart kernels; the host only reads the 16-byte
// status word between graph launches, pipelined one batch behind.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <thread>
#include <vector>

#include "pdlp.h"
#include "pdlp_dev.h"

namespace pdlp {
void launch_primal(const Params& p, hipStream_t s);
void launch_dual(const Params& p, hipStream_t s);
void launch_decide(const Params& p, hipStream_t s);
void launch_eval(const Params& p, hipStream_t s);
void launch_init(const Params& p, const double* xs, const double* ys, hipStream_t s);
void launch_output(const Params& p, hipStream_t s);
void launch_set_limit(DevState* st, int status, hipStream_t s);
void set_pass_events(hipEvent_t t0, hipEvent_t t1);
void launch_batch(const Params& p, const BatchParams& bp, int grid, hipStream_t s);
int batch_occupancy(size_t lds_bytes);
size_t batch_lds_bytes(const BatchParams& bp);
hipError_t batch_prepare(size_t lds_bytes);
int batch_tile();
int batch_static_lds();
void launch_seg_sumsq(int nlp, const int32_t* off, const double* a, double* out, int stride, int slot, hipStream_t s);
void launch_seg_absmax(int nlp, const int32_t* row_off, const int32_t* rp, const double* v, double* out,
                       hipStream_t s);
hipError_t setup_normalize(int m, const int32_t* rp, double* v, const double* b, const int8_t* rt, double* q,
                           int8_t* ineq, int8_t* le, int32_t* rowid, hipStream_t s);
hipError_t setup_transpose(int m, int n, int64_t nnz, const int32_t* ci, const double* v, const int32_t* rowid,
                           int32_t* rpT, int32_t* ciT, double* vT, int32_t* rowidT, int32_t* perm_out,
                           hipStream_t s);
hipError_t setup_scale(int m, int n, int64_t nnz, const int32_t* rp, const int32_t* ci, const int32_t* rowid,
                       double* v, const int32_t* rpT, const int32_t* ciT, const int32_t* rowidT, double* vT,
                       int ruiz, double alpha, double* D1, double* D2, double* d1, double* d2, hipStream_t s);
hipError_t setup_vectors(int m, int n, const double* D1, const double* D2, const double* c0, const double* l0,
                         const double* u0, double* c, double* l, double* u, double* q, hipStream_t s);
hipError_t setup_sumsq(int64_t n, const double* a, double* part, double* out, hipStream_t s);
hipError_t setup_absmax(int64_t nnz, const double* v, unsigned long long* out, hipStream_t s);
hipError_t setup_to_f32(int64_t nnz, const double* v, float* f, hipStream_t s);
hipError_t setup_fill(int64_t n, double* a, double val, hipStream_t s);
hipError_t setup_permute_values(int64_t count, const int32_t* perm, const double* v, const float* vf, double* pv,
                                float* pvf, hipStream_t s);
hipError_t setup_permute(int64_t nnz, const int32_t* perm, const int32_t* ci, const double* v, const float* vf,
                         int32_t* pci, double* pv, float* pvf, hipStream_t s);
hipError_t setup_rename(int64_t nnz, const int32_t* inv, int32_t* ci, hipStream_t s);
hipError_t setup_gather_rows(int32_t m, const int32_t* perm, const double* src, double* dst, hipStream_t s);
hipError_t setup_gather_rows_i8(int32_t m, const int32_t* perm, const int8_t* src, int8_t* dst, hipStream_t s);
}  // namespace pdlp

using namespace pdlp;

namespace {

thread_local std::string g_create_error = "no error";

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct HipFail {
  hipError_t e;
  const char* what;
};

inline void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw HipFail{e, what};
}

// Row-block partition of a CSR-like structure (see RowBlock) over rows
// [begin, end): every row longer than `tile` becomes a block of its own, listed
// first so that these heavier blocks are dispatched before the short ones; the
// runs of short rows between them are cut greedily at `tile` nonzeros or
// kMaxRows rows.
std::vector<RowBlock> partition_rows(const int32_t* rp, int begin, int end, int tile = kTile,
                                     int max_rows = kMaxRows) {
  std::vector<RowBlock> longs, shorts;
  int r = begin;
  while (r < end) {
    if (rp[r + 1] - rp[r] > tile) {
      longs.push_back(RowBlock{r, r + 1});
      ++r;
      continue;
    }
    const int r0 = r;
    int nz = 0;
    while (r < end && r - r0 < max_rows) {
      const int len = rp[r + 1] - rp[r];
      if (len > tile || nz + len > tile) break;
      nz += len;
      ++r;
    }
    shorts.push_back(RowBlock{r0, r});
  }
  longs.insert(longs.end(), shorts.begin(), shorts.end());
  return longs;
}

std::vector<RowBlock> partition_rows(const int32_t* rp, int nrows) {
  std::vector<RowBlock> b = partition_rows(rp, 0, nrows);
  if (b.empty()) b.push_back(RowBlock{0, 0});
  return b;
}

// Column-panel layout (see PanelCsr), built on the host from the structure.
struct HostPanels {
  std::vector<int32_t> seg_ptr, slot_seg, row_seg, perm;
  std::vector<RowBlock> sblocks, sblocks_wide;   // phase-1 blocks of kTile and of kTileWide nonzeros
};

// Rows [r0, nrows) with at least min_len nonzeros only (the others get no
// segments); seg_ptr offsets count over those rows' nonzeros, perm holds CSR
// indices.
HostPanels build_panels(const int32_t* rp, const int32_t* ci, int nrows, int ncols, const int32_t* col_ptr,
                        int r0 = 0, int min_len = 0) {
  HostPanels H;
  auto in = [&](int r) { return rp[r + 1] - rp[r] >= min_len; };
  int64_t nnz = 0;
  for (int r = r0; r < nrows; ++r)
    if (in(r)) nnz += rp[r + 1] - rp[r];
  // panel boundaries: about nnz / kPanels nonzeros of these rows each
  // (col_ptr = row pointer of the transpose when the range is every row;
  // otherwise the range's own column counts)
  std::vector<int32_t> own;
  if (r0 > 0 || min_len > 0 || !col_ptr) {
    own.assign((size_t)ncols + 1, 0);
    for (int r = r0; r < nrows; ++r)
      if (in(r))
        for (int32_t e = rp[r]; e < rp[r + 1]; ++e) own[(size_t)ci[e] + 1]++;
    for (int j = 0; j < ncols; ++j) own[(size_t)j + 1] += own[(size_t)j];
    col_ptr = own.data();
  }
  std::vector<int32_t> cb(kPanels + 1, ncols);
  cb[0] = 0;
  for (int p = 1, j = 0; p < kPanels; ++p) {
    const int64_t target = nnz * p / kPanels;
    while (j < ncols && col_ptr[j] < target) ++j;
    cb[p] = j;
  }
  std::vector<uint8_t> colpan((size_t)ncols);
  for (int p = 0; p < kPanels; ++p)
    for (int j = cb[p]; j < cb[p + 1]; ++j) colpan[(size_t)j] = (uint8_t)p;
  std::vector<uint8_t> mask((size_t)nrows, 0);
  std::vector<int64_t> pnnz(kPanels, 0), pseg(kPanels, 0);
  for (int r = r0; r < nrows; ++r) {
    if (!in(r)) continue;
    for (int32_t e = rp[r]; e < rp[r + 1]; ++e) {
      const int p = colpan[(size_t)ci[e]];
      mask[(size_t)r] |= (uint8_t)(1u << p);
      pnnz[p]++;
    }
    for (int p = 0; p < kPanels; ++p) pseg[p] += (mask[(size_t)r] >> p) & 1;
  }
  H.row_seg.assign((size_t)nrows + 1, 0);
  for (int r = 0; r < nrows; ++r) H.row_seg[(size_t)r + 1] = H.row_seg[(size_t)r] + __builtin_popcount(mask[(size_t)r]);
  const int nseg = H.row_seg[(size_t)nrows];
  std::vector<int64_t> ent(kPanels), seg(kPanels);
  int64_t eo = 0, so = 0;
  for (int p = 0; p < kPanels; ++p) {
    ent[p] = eo;
    seg[p] = so;
    eo += pnnz[p];
    so += pseg[p];
  }
  std::vector<int64_t> seg_base(seg);
  H.seg_ptr.assign((size_t)nseg + 1, 0);
  H.slot_seg.assign((size_t)nseg, 0);
  H.perm.assign((size_t)nnz, 0);
  std::vector<int32_t> last(kPanels, -1);
  for (int r = r0; r < nrows; ++r) {
    if (!in(r)) continue;
    for (int32_t e = rp[r]; e < rp[r + 1]; ++e) {
      const int p = colpan[(size_t)ci[e]];
      if (last[p] != r) {
        const int64_t sp = seg[p]++;
        H.seg_ptr[(size_t)sp] = (int32_t)ent[p];
        H.slot_seg[(size_t)(H.row_seg[(size_t)r] + __builtin_popcount(mask[(size_t)r] & ((1u << p) - 1u)))] =
            (int32_t)sp;
        last[p] = r;
      }
      H.perm[(size_t)ent[p]++] = e;
    }
  }
  H.seg_ptr[(size_t)nseg] = (int32_t)nnz;
  // phase-1 blocks of each panel, interleaved so that block i serves panel i % kPanels
  for (int tile : {kTile, kTileWide}) {
    std::vector<std::vector<RowBlock>> pb(kPanels);
    size_t nbmax = 0;
    for (int p = 0; p < kPanels; ++p) {
      pb[p] = partition_rows(H.seg_ptr.data(), (int)seg_base[p], (int)(seg_base[p] + pseg[p]), tile);
      nbmax = std::max(nbmax, pb[p].size());
    }
    if (nbmax == 0) nbmax = 1;
    std::vector<RowBlock>& sb = tile == kTile ? H.sblocks : H.sblocks_wide;
    sb.assign(nbmax * kPanels, RowBlock{0, 0});
    for (int p = 0; p < kPanels; ++p)
      for (size_t j = 0; j < pb[p].size(); ++j) sb[j * kPanels + p] = pb[p][j];
  }
  return H;
}

// LDS-staged panel layout (see StagedCsr), built on the host from the
// structure.  Rows [0, rlong) -- the leading rows with at least `min_len`
// nonzeros -- are cut into panels of kStageWidth columns; each panel's
// segments are sorted by length (longest first, then by row), numbered in
// that order and grouped in chunks of kStageLanes, stored lane-interleaved
// with zero padding up to the chunk's longest segment.  The panels' chunks
// are cut into at most `items` work items (one per CU: a single wave), each
// panel into runs of about equal entry counts, as many per panel as the
// smallest item size allows -- so panels of unequal weight (columns of
// unequal counts) still give items of about equal work.  The rows [rlong,
// nrows) go through column panels of their own (build_panels from rlong).
struct HostStaged {
  int32_t rlong = 0, nseg = 0;
  int64_t nnz_long = 0, nent = 0;
  int32_t npan = 0;
  std::vector<int32_t> wpanel, wchunk, coff, clen, cseg, perm, srow;
  std::vector<uint16_t> pci;   // column relative to the panel (kStageWidth <= 65536)
};

constexpr int kStageMinLen = 256;   // nonzeros of a row summed through the staged panels

// Nonzeros of the leading rows with at least min_len nonzeros.
int64_t leading_long_nnz(const int32_t* rp, int nrows, int min_len) {
  int r = 0;
  while (r < nrows && rp[r + 1] - rp[r] >= min_len) ++r;
  return (int64_t)rp[r] - rp[0];
}

HostStaged build_staged(const int32_t* rp, const int32_t* ci, int nrows, int ncols, int min_len, int items) {
  HostStaged H;
  int rl = 0;
  while (rl < nrows && rp[rl + 1] - rp[rl] >= min_len) ++rl;
  H.rlong = rl;
  H.nnz_long = (int64_t)rp[rl] - rp[0];
  const int np = (ncols + kStageWidth - 1) / kStageWidth;
  // segments (nonzero count, row) of every panel
  struct Seg {
    int32_t cnt, row;
  };
  std::vector<std::vector<Seg>> ps((size_t)np);
  std::vector<int32_t> cnt((size_t)np, 0), touched;
  for (int r = 0; r < rl; ++r) {
    touched.clear();
    for (int32_t e = rp[r]; e < rp[r + 1]; ++e) {
      const int p = ci[e] / kStageWidth;
      if (cnt[(size_t)p]++ == 0) touched.push_back(p);
    }
    for (int p : touched) {
      ps[(size_t)p].push_back(Seg{cnt[(size_t)p], r});
      cnt[(size_t)p] = 0;
    }
  }
  // ids: panel-major, longest first inside a panel; chunks of kStageLanes
  std::vector<int64_t> sbase((size_t)np + 1, 0);
  for (int p = 0; p < np; ++p) {
    std::stable_sort(ps[(size_t)p].begin(), ps[(size_t)p].end(),
                     [](const Seg& a, const Seg& b) { return a.cnt > b.cnt; });
    sbase[(size_t)p + 1] = sbase[(size_t)p] + (int64_t)ps[(size_t)p].size();
  }
  H.nseg = (int32_t)sbase[(size_t)np];
  std::vector<int64_t> seg_at((size_t)H.nseg);   // entry position of a segment's first nonzero
  std::vector<int32_t> chunk0((size_t)np + 1, 0);
  int64_t ent = 0;
  for (int p = 0; p < np; ++p) {
    chunk0[(size_t)p] = (int32_t)H.coff.size();
    const std::vector<Seg>& v = ps[(size_t)p];
    for (size_t i = 0; i < v.size(); i += kStageLanes) {
      const int32_t len = v[i].cnt;
      H.coff.push_back((int32_t)ent);
      H.clen.push_back(len);
      H.cseg.push_back((int32_t)(sbase[(size_t)p] + (int64_t)i));
      for (size_t l = 0; l < (size_t)kStageLanes && i + l < v.size(); ++l)
        seg_at[(size_t)(sbase[(size_t)p] + (int64_t)(i + l))] = ent + (int64_t)l;
      ent += (int64_t)kStageLanes * len;
    }
  }
  chunk0[(size_t)np] = (int32_t)H.coff.size();
  H.cseg.push_back(H.nseg);
  H.nent = ent;
  // each segment's row; every long row's entries in place (segments in panel order)
  H.npan = np;
  H.srow.assign((size_t)std::max(H.nseg, 1), 0);
  std::vector<std::vector<int32_t>> rowsegs((size_t)rl);
  for (int p = 0; p < np; ++p)
    for (size_t i = 0; i < ps[(size_t)p].size(); ++i) {
      const int32_t sid = (int32_t)(sbase[(size_t)p] + (int64_t)i);
      rowsegs[(size_t)ps[(size_t)p][i].row].push_back(sid);
      H.srow[(size_t)sid] = ps[(size_t)p][i].row;
    }
  H.perm.assign((size_t)std::max<int64_t>(ent, 1), -1);
  H.pci.assign((size_t)std::max<int64_t>(ent, 1), 0);
  std::vector<int64_t> at((size_t)np);
  for (int r = 0; r < rl; ++r) {
    for (int32_t sid : rowsegs[(size_t)r]) {
      const int p = (int)(std::upper_bound(sbase.begin(), sbase.end(), (int64_t)sid) - sbase.begin()) - 1;
      at[(size_t)p] = seg_at[(size_t)sid];
    }
    for (int32_t e = rp[r]; e < rp[r + 1]; ++e) {
      const int p = ci[e] / kStageWidth;
      const int64_t pos = at[(size_t)p];
      at[(size_t)p] += kStageLanes;
      H.perm[(size_t)pos] = e;
      H.pci[(size_t)pos] = (uint16_t)(ci[e] - p * kStageWidth);
    }
  }
  // work items: the smallest item size T whose per-panel item counts
  // ceil(entries / T) (at most one per chunk) add up to at most `cap`; each
  // panel's chunks are then cut into that many runs of about equal entries
  std::vector<int64_t> ptot((size_t)np, 0);
  for (int p = 0; p < np; ++p) {
    const int32_t a = chunk0[(size_t)p], b = chunk0[(size_t)p + 1];
    if (a < b) ptot[(size_t)p] = (b < (int32_t)H.coff.size() ? (int64_t)H.coff[(size_t)b] : ent) - H.coff[(size_t)a];
  }
  auto count_for = [&](int64_t T, int p) {
    const int64_t nc = chunk0[(size_t)p + 1] - chunk0[(size_t)p];
    return std::min<int64_t>(nc, (ptot[(size_t)p] + T - 1) / T);
  };
  struct Item {
    int32_t p, a, b;   // panel, chunk range
  };
  auto cut = [&](int cap) {
    int64_t lo = 1, hi = std::max<int64_t>(ent, 1);
    while (lo < hi) {
      const int64_t T = lo + (hi - lo) / 2;
      int64_t tot_items = 0;
      for (int p = 0; p < np; ++p) tot_items += count_for(T, p);
      if (tot_items <= std::max(cap, np)) hi = T;
      else lo = T + 1;
    }
    std::vector<Item> it;
    for (int p = 0; p < np; ++p) {
      const int32_t a = chunk0[(size_t)p], b = chunk0[(size_t)p + 1];
      if (a == b) continue;
      const int64_t e0 = H.coff[(size_t)a];
      const int64_t tot = ptot[(size_t)p];
      const int64_t per_panel = std::max<int64_t>(1, count_for(lo, p));
      int64_t k = 1;
      int32_t start = a;
      for (int32_t c = a; c < b; ++c) {
        const int64_t done = (int64_t)H.coff[(size_t)c] - e0 + (int64_t)kStageLanes * H.clen[(size_t)c];
        if (c + 1 == b || (k < per_panel && done * per_panel >= tot * k)) {
          it.push_back(Item{p, start, c + 1});
          start = c + 1;
          ++k;
        }
      }
    }
    return it;
  };
  // workgroups are dispatched round-robin over the 8 XCDs (workgroup i on
  // XCD i % 8): all items of a panel go to one XCD, whose L2 then gathers
  // that panel's segment-sum stores (the panels dealt to the XCDs by item
  // count, largest first); slot 8k + x holds XCD x's k-th item, empty
  // slots pad the shorter queues, at most `items` slots in all
  std::vector<std::vector<Item>> q(8);
  for (int cap = std::max(items, 8);; cap -= 8) {
    const std::vector<Item> it = cut(cap);
    std::vector<int> cnt_p((size_t)np, 0), order;
    for (const Item& x : it) cnt_p[(size_t)x.p]++;
    for (int p = 0; p < np; ++p)
      if (cnt_p[(size_t)p]) order.push_back(p);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cnt_p[(size_t)a] > cnt_p[(size_t)b]; });
    std::vector<int> bin((size_t)np, 0), load(8, 0);
    for (int p : order) {
      const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      bin[(size_t)p] = x;
      load[(size_t)x] += cnt_p[(size_t)p];
    }
    for (auto& v : q) v.clear();
    for (const Item& x : it) q[(size_t)bin[(size_t)x.p]].push_back(x);
    const int mx = *std::max_element(load.begin(), load.end());
    if (8 * mx <= std::max(items, 8) || cap <= 8) break;
  }
  size_t depth = 0;
  for (const auto& v : q) depth = std::max(depth, v.size());
  for (size_t k = 0; k < depth; ++k)
    for (int x = 0; x < 8; ++x) {
      const Item e = k < q[(size_t)x].size() ? q[(size_t)x][k] : Item{0, 0, 0};
      H.wpanel.push_back(e.p);
      H.wchunk.push_back(e.a);
      H.wchunk.push_back(e.b);
    }
  return H;
}

}  // namespace

struct pdlp_handle {
  int32_t m = 0, n = 0;
  int64_t nnz = 0;
  pdlp_options opt{};
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  std::vector<void*> dev_allocs;
  std::vector<void*> host_allocs;
  Params P{};
  int32_t *rp = nullptr, *ci = nullptr, *rowid = nullptr, *rpT = nullptr, *ciT = nullptr, *rowidT = nullptr,
          *perm = nullptr;
  double *val = nullptr, *valT = nullptr;
  float *valf = nullptr, *valTf = nullptr;
  double *c0 = nullptr, *l0 = nullptr, *u0 = nullptr, *b0 = nullptr;
  double *c = nullptr, *l = nullptr, *u = nullptr, *q = nullptr, *D1 = nullptr, *D2 = nullptr;
  int8_t *rt = nullptr, *ineq = nullptr, *le = nullptr;
  double *xo = nullptr, *yo = nullptr, *rco = nullptr;
  double *wx = nullptr, *wy = nullptr;
  bool has_warm = false;
  double warm_omega = 0.0;
  DevState* st = nullptr;
  DevState* st_host[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // the short graph for the end of a step budget: kTailSlots attempt slots
  // and an evaluation, so that a solve with max_iter ends with few idle slots
  hipGraph_t graph_tail = nullptr;
  hipGraphExec_t gexec_tail = nullptr;
  int slots_per_round = 0, rounds = 0;
  double eta0 = 1.0, omega0 = 1.0;
  double probe_ms[2] = {0.0, 0.0};
  DevState* probe_st = nullptr;   // the private state of the layout timing
  int32_t persist_grid = 2048;   // persistent grid of the row-block kernels (CUs x 8, a multiple of 8)
  // the kTileWide tilings of K and K' (row blocks, panel phase-1 blocks) a step view may take
  const RowBlock* wide_blocks[2] = {nullptr, nullptr};
  int32_t wide_nblocks[2] = {0, 0};
  const RowBlock* wide_sblocks[2] = {nullptr, nullptr};
  int32_t wide_nsblocks[2] = {0, 0};
  // the LDS-staged layouts of K and K' a step view may take
  StagedCsr stg[2] = {};
  PanelCsr stg_pan[2] = {};   // the staged step views' column panels of the short rows
  bool has_stg[2] = {false, false};
  SellCsr sel[2] = {};
  bool has_sel[2] = {false, false};
  // device of the handle, and the sizes (doubles) of the reduction partials
  // that pdlp_solve_noalloc places in the static scratch
  int device = 0;
  size_t red_k = 0, red_t = 0;
  std::string err = "no error";
  bool solved = false;
  pdlp_info info{};
  double setup_s = 0.0;
  // batch handles (count > 0): LP b owns rows [row_off[b], row_off[b+1]) and
  // columns [col_off[b], col_off[b+1]) of the packed block-diagonal problem
  int32_t count = 0;
  std::vector<int32_t> row_off_h, col_off_h;
  std::vector<int64_t> nnz_h;
  std::vector<uint8_t> lanes_h;
  std::vector<int8_t> warm_h;
  std::vector<double> omega_warm_h;
  std::vector<DevState> bst_h;
  int32_t grid = 0;
  int32_t *row_off = nullptr, *col_off = nullptr, *order = nullptr;
  int32_t* order2 = nullptr;   // queue order of a relaunch over paused LPs
  uint8_t* lanes = nullptr;
  RowBlock *bk = nullptr, *bt = nullptr;
  int32_t *bk_off = nullptr, *bt_off = nullptr;
  int8_t* warm = nullptr;
  double *norms = nullptr, *kmax = nullptr, *omega_warm = nullptr;
  DevState* bst = nullptr;
  uint32_t* queue = nullptr;
  uint64_t* t0 = nullptr;
  double tick_hz = 0.0;
  int32_t lds_m = 0, lds_n = 0;   // LDS room for an LP's vectors and row pointers in the batched kernel
  int32_t lds_bk = 0, lds_bt = 0; // ... and its block descriptors
  int32_t max_bk = 0, max_bt = 0; // most row blocks of one LP
  size_t lds_bytes = 0;
  // hand-off: every LP's row blocks in the single-LP tiling (kTile), and the
  // streams on which LPs paused by the persistent launch are finished
  RowBlock *hk = nullptr, *ht = nullptr;
  std::vector<int32_t> hk_off, ht_off;
  int32_t max_hk = 1, max_ht = 1;
  std::vector<double> norms_h;
  std::vector<int64_t> handoff_h;
  struct Lane {
    hipStream_t s = nullptr;
    double *pa = nullptr, *pb = nullptr, *pe0 = nullptr, *pe1 = nullptr, *pe2 = nullptr, *pe3 = nullptr,
           *pe4 = nullptr, *pg = nullptr;
    DevState* hst[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
  };
  std::vector<Lane> lanes_ho;
  // presolve (single-LP handles): the device holds the reduced LP; orig is the
  // user's LP for the postsolve and the warm-start mapping
  bool presolved = false;
  Presolve pre;
  HostLP orig;
  // row renumbering (single-LP handles, row_order = 1): device row r is row
  // rperm[r] of the LP given to the device (empty: the identity); rp_given and
  // rp_dev are K's row pointers in the two numberings
  std::vector<int32_t> rperm, rp_given, rp_dev;
  // column renumbering (single-LP handles, row_order = 2, or 1 on large LPs):
  // device column j is column cperm[j] of the LP given to the device (empty:
  // the identity)
  std::vector<int32_t> cperm;

  // device row order <-> the given order, for vectors over the rows
  void rows_to_given(const double* dev, double* given) const {
    for (size_t r = 0; r < rperm.size(); ++r) given[rperm[r]] = dev[r];
  }
  void rows_to_dev(const double* given, double* dev) const {
    for (size_t r = 0; r < rperm.size(); ++r) dev[r] = given[rperm[r]];
  }
  // device column order <-> the given order, for vectors over the columns
  void cols_to_given(const double* dev, double* given) const {
    for (size_t j = 0; j < cperm.size(); ++j) given[cperm[j]] = dev[j];
  }
  void cols_to_dev(const double* given, double* dev) const {
    for (size_t j = 0; j < cperm.size(); ++j) dev[j] = given[cperm[j]];
  }

  template <typename T>
  T* dalloc(size_t count) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) throw HipFail{e, "hipMalloc"};
    dev_allocs.push_back(p);
    e = hipMemsetAsync(p, 0, bytes, stream);
    if (e != hipSuccess) throw HipFail{e, "hipMemsetAsync"};
    return static_cast<T*>(p);
  }

  void release() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    if (gexec_tail) (void)hipGraphExecDestroy(gexec_tail);
    if (graph_tail) (void)hipGraphDestroy(graph_tail);
    gexec = nullptr;
    graph = nullptr;
    gexec_tail = nullptr;
    graph_tail = nullptr;
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e), e = nullptr;
    for (Lane& L : lanes_ho) {
      if (L.s) (void)hipStreamSynchronize(L.s);
      for (auto& e : L.ev)
        if (e) (void)hipEventDestroy(e), e = nullptr;
      if (L.s) (void)hipStreamDestroy(L.s);
      L.s = nullptr;
    }
    lanes_ho.clear();
    if (stream) (void)hipStreamSynchronize(stream);
    for (void* p : dev_allocs) (void)hipFree(p);
    dev_allocs.clear();
    for (void* p : host_allocs) (void)hipHostFree(p);
    host_allocs.clear();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    cap_stream = nullptr;
  }
};

static int fail(pdlp_handle* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  else g_create_error = msg;
  return code;
}

static std::string hip_msg(const HipFail& f) {
  return std::string(f.what) + ": " + hipGetErrorString(f.e);
}

extern "C" int pdlp_default_options(pdlp_options* o) {
  if (!o) return PDLP_ERR_ARG;
  o->eps_rel = 1e-4;
  o->max_iter = 1000000;
  o->time_limit_s = 3600.0;
  o->eval_period = 64;
  o->ruiz_iters = 10;
  o->pc_alpha = 1.0;
  o->pw_theta = 0.5;
  o->eps_zero = 1e-10;
  o->beta_suff = 0.2;
  o->beta_nec = 0.8;
  o->beta_art = 0.36;
  o->a_precision = PDLP_A_FP64;
  o->kkt_omega_power = 2;
  o->trace = 0;
  o->poll_every = 1;
  o->graph = 1;
  o->spmv_layout = -1;
  o->spmv_layout_kt = -2;
  o->batch_lanes = 0;
  o->batch_grid = 0;
  o->batch_handoff = 2048;
  o->handoff_streams = 8;
  o->detect_infeas = 1;
  o->eps_infeas = 1e-8;
  o->infeas_every = 4;
  o->presolve = 0;
  o->restart_metric = 0;
  o->row_order = 1;
  return PDLP_OK;
}

static int check_options(const pdlp_options& o, std::string& why) {
  if (!(o.eps_rel >= 0.0) || !std::isfinite(o.eps_rel)) return why = "eps_rel must be finite and >= 0", -1;
  if (o.max_iter < 0) return why = "max_iter must be >= 0", -1;
  if (!(o.time_limit_s > 0.0)) return why = "time_limit_s must be > 0", -1;
  if (o.eval_period < 1 || o.eval_period > 1024) return why = "eval_period must be in [1, 1024]", -1;
  if (o.ruiz_iters < 0 || o.ruiz_iters > 1000) return why = "ruiz_iters must be in [0, 1000]", -1;
  if (!(o.pc_alpha <= 2.0) || std::isnan(o.pc_alpha)) return why = "pc_alpha must be <= 2", -1;
  if (!(o.pw_theta >= 0.0 && o.pw_theta <= 1.0)) return why = "pw_theta must be in [0, 1]", -1;
  if (!(o.eps_zero >= 0.0) || !std::isfinite(o.eps_zero)) return why = "eps_zero must be finite and >= 0", -1;
  if (!(o.beta_suff > 0.0 && o.beta_nec > 0.0 && o.beta_art > 0.0)) return why = "restart betas must be > 0", -1;
  if (o.a_precision != PDLP_A_FP64 && o.a_precision != PDLP_A_FP32) return why = "a_precision must be 0 or 1", -1;
  if (o.kkt_omega_power != 1 && o.kkt_omega_power != 2) return why = "kkt_omega_power must be 1 or 2", -1;
  if (o.trace < 0) return why = "trace must be >= 0", -1;
  if (o.poll_every < 1) return why = "poll_every must be >= 1", -1;
  if (o.graph != 0 && o.graph != 1) return why = "graph must be 0 or 1", -1;
  // -1; 0, 1, 2 plus 4 and/or 8; 3, 19, 35 (LDS-staged step passes, phase-1 workgroups of 256, 512, 1024);
  // 64, 80, 96 (SELL-64 step passes)
  auto bad_layout = [](int v) {
    if (v == 3 || v == 19 || v == 35 || v == 64 || v == 80 || v == 96) return false;
    return v < -1 || v > 14 || (v >= 0 && (v & 3) == 3);
  };
  if (bad_layout(o.spmv_layout))
    return why = "spmv_layout must be -1, or 0, 1, 2 plus 4 (persistent grid) and/or 8 (wide step tiles), "
                 "or 3, 19, 35 (LDS-staged step passes), or 64, 80, 96 (SELL-64 step passes)", -1;
  if (o.spmv_layout_kt != -2 && bad_layout(o.spmv_layout_kt))
    return why = "spmv_layout_kt must be -2, -1, or 0, 1, 2 plus 4 (persistent grid) and/or 8 (wide step tiles), "
                 "or 3, 19, 35 (LDS-staged step passes), or 64, 80, 96 (SELL-64 step passes)", -1;
  if (o.batch_lanes < -1 || o.batch_lanes > 64 || (o.batch_lanes > 0 && (o.batch_lanes & (o.batch_lanes - 1))))
    return why = "batch_lanes must be -1, 0 or a power of two up to 64", -1;
  if (o.batch_grid < 0) return why = "batch_grid must be >= 0", -1;
  if (o.batch_handoff < 0) return why = "batch_handoff must be >= 0", -1;
  if (o.handoff_streams < 1 || o.handoff_streams > 16) return why = "handoff_streams must be in 1..16", -1;
  if (o.detect_infeas != 0 && o.detect_infeas != 1) return why = "detect_infeas must be 0 or 1", -1;
  if (!(o.eps_infeas > 0.0) || !std::isfinite(o.eps_infeas)) return why = "eps_infeas must be finite and > 0", -1;
  if (o.infeas_every < 1) return why = "infeas_every must be >= 1", -1;
  if (o.presolve != 0 && o.presolve != 1) return why = "presolve must be 0 or 1", -1;
  if (o.restart_metric != 0 && o.restart_metric != 1) return why = "restart_metric must be 0 or 1", -1;
  if (o.row_order < 0 || o.row_order > 2) return why = "row_order must be 0, 1 or 2", -1;
  return 0;
}

// Host-side validation of the LP (arrays on the host).
static int validate(int32_t m, int32_t n, int64_t nnz, const int32_t* rp, const int32_t* ci, const double* v,
                    const double* c, const double* b, const double* l, const double* u, const int8_t* rt,
                    std::string& why) {
  char buf[256];
  if (rp[0] != 0) return why = "row_ptr[0] must be 0", -1;
  for (int32_t i = 0; i < m; ++i)
    if (rp[i + 1] < rp[i]) {
      snprintf(buf, sizeof buf, "row_ptr decreases at row %d", i);
      return why = buf, -1;
    }
  if ((int64_t)rp[m] != nnz) return why = "row_ptr[m] != nnz", -1;
  std::vector<int32_t> mark((size_t)n, -1);
  for (int32_t i = 0; i < m; ++i) {
    for (int32_t p = rp[i]; p < rp[i + 1]; ++p) {
      const int32_t j = ci[p];
      if (j < 0 || j >= n) {
        snprintf(buf, sizeof buf, "col_idx[%d] = %d out of range [0, %d)", p, j, n);
        return why = buf, -1;
      }
      if (mark[(size_t)j] == i) {
        snprintf(buf, sizeof buf, "duplicate column %d in row %d", j, i);
        return why = buf, -1;
      }
      mark[(size_t)j] = i;
      if (!std::isfinite(v[p])) {
        snprintf(buf, sizeof buf, "val[%d] is not finite", p);
        return why = buf, -1;
      }
    }
    if (!std::isfinite(b[i])) {
      snprintf(buf, sizeof buf, "b[%d] is not finite", i);
      return why = buf, -1;
    }
    if (rt[i] < 0 || rt[i] > 2) {
      snprintf(buf, sizeof buf, "row_type[%d] = %d is not EQ/GE/LE", i, (int)rt[i]);
      return why = buf, -1;
    }
  }
  for (int32_t j = 0; j < n; ++j) {
    if (!std::isfinite(c[j])) {
      snprintf(buf, sizeof buf, "c[%d] is not finite", j);
      return why = buf, -1;
    }
    if (std::isnan(l[j]) || std::isnan(u[j]) || l[j] == INFINITY || u[j] == -INFINITY || l[j] > u[j]) {
      snprintf(buf, sizeof buf, "bounds of x[%d] are invalid (l=%g, u=%g)", j, l[j], u[j]);
      return why = buf, -1;
    }
  }
  return 0;
}

template <typename T>
static void fetch(std::vector<T>& dst, const T* src, size_t count, int mem) {
  dst.resize(std::max<size_t>(count, 1));
  if (count == 0) return;
  if (mem == PDLP_MEM_HOST) std::memcpy(dst.data(), src, count * sizeof(T));
  else check(hipMemcpy(dst.data(), src, count * sizeof(T), hipMemcpyDeviceToHost), "hipMemcpy(D2H) of the problem");
}

constexpr int kTailSlots = 8;   // attempt slots of the short graph

static void build_graph(pdlp_handle* h) {
  const int P = h->opt.eval_period;
  h->slots_per_round = P + std::max(2, P / 8);
  h->rounds = std::max(1, 64 / P);
  check(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  for (int r = 0; r < h->rounds; ++r) {
    for (int s = 0; s < h->slots_per_round; ++s) {
      launch_primal(h->P, h->cap_stream);
      launch_dual(h->P, h->cap_stream);
      launch_decide(h->P, h->cap_stream);
    }
    launch_eval(h->P, h->cap_stream);
  }
  check(hipStreamEndCapture(h->cap_stream, &h->graph), "hipStreamEndCapture");
  check(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  check(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  for (int s = 0; s < kTailSlots; ++s) {
    launch_primal(h->P, h->cap_stream);
    launch_dual(h->P, h->cap_stream);
    launch_decide(h->P, h->cap_stream);
  }
  launch_eval(h->P, h->cap_stream);
  check(hipStreamEndCapture(h->cap_stream, &h->graph_tail), "hipStreamEndCapture");
  check(hipGraphInstantiate(&h->gexec_tail, h->graph_tail, nullptr, nullptr, 0), "hipGraphInstantiate");
}

static int elem_grid(int n) {
  int g = (n + kBlock - 1) / kBlock;
  if (g > kElemBlocks) g = kElemBlocks;
  return g < 1 ? 1 : g;
}

// SELL-64 layout (see SellCsr), built on the host from the structure: chunk c
// holds rows [64c, 64c + 64) lane-interleaved, zero-padded to its longest
// row.  perm holds CSR indices (-1 on padding).  nent = -1: the entries would
// not fit 32-bit offsets.
struct HostSell {
  int64_t nent = 0;
  std::vector<int32_t> coff, clen, perm, sci;
};

HostSell build_sell(const int32_t* rp, const int32_t* ci, int nrows) {
  HostSell H;
  const int nch = (nrows + 63) / 64;
  H.coff.resize((size_t)nch);
  H.clen.resize((size_t)nch);
  int64_t ent = 0;
  for (int c = 0; c < nch; ++c) {
    int32_t len = 0;
    for (int r = 64 * c; r < std::min(nrows, 64 * c + 64); ++r) len = std::max(len, rp[r + 1] - rp[r]);
    H.coff[(size_t)c] = (int32_t)std::min<int64_t>(ent, INT32_MAX);
    H.clen[(size_t)c] = len;
    ent += (int64_t)64 * len;
  }
  if (ent >= ((int64_t)1 << 31)) {
    H.nent = -1;
    return H;
  }
  H.nent = ent;
  H.perm.assign((size_t)std::max<int64_t>(ent, 1), -1);
  H.sci.assign((size_t)std::max<int64_t>(ent, 1), 0);
  for (int r = 0; r < nrows; ++r) {
    const int64_t at = H.coff[(size_t)(r / 64)] + (r % 64);
    for (int32_t k = 0; k < rp[r + 1] - rp[r]; ++k) {
      H.perm[(size_t)(at + 64 * k)] = rp[r] + k;
      H.sci[(size_t)(at + 64 * k)] = ci[rp[r] + k];
    }
  }
  return H;
}

// Device copy of a SELL-64 layout for the step view of matrix `which`, whose
// step pass gathers a vector of `ngathered` entries (kept in h->sel until the
// chooser or the option selects it).
static void upload_sell(pdlp_handle* h, int which, const HostSell& H, int ngathered, const double* v,
                        const float* vf) {
  hipStream_t s = h->stream;
  const hipMemcpyKind kind = hipMemcpyHostToDevice;
  SellCsr& S = h->sel[which];
  S = SellCsr{};
  S.nchunks = (int32_t)H.coff.size();
  S.hot = std::min(kSellHot, ngathered);
  int32_t* coff = h->dalloc<int32_t>(H.coff.size());
  int32_t* clen = h->dalloc<int32_t>(H.clen.size());
  const int64_t ne = std::max<int64_t>(H.nent, 1);
  int32_t* sci = h->dalloc<int32_t>((size_t)ne);
  int32_t* perm = h->dalloc<int32_t>((size_t)ne);
  double* sv = h->dalloc<double>((size_t)ne);
  float* svf = vf ? h->dalloc<float>((size_t)ne) : nullptr;
  if (!H.coff.empty()) {
    check(hipMemcpyAsync(coff, H.coff.data(), H.coff.size() * 4, kind, s), "upload sell");
    check(hipMemcpyAsync(clen, H.clen.data(), H.clen.size() * 4, kind, s), "upload sell");
  }
  if (H.nent > 0) {
    check(hipMemcpyAsync(sci, H.sci.data(), (size_t)H.nent * 4, kind, s), "upload sell");
    check(hipMemcpyAsync(perm, H.perm.data(), (size_t)H.nent * 4, kind, s), "upload sell");
    check(setup_permute_values(H.nent, perm, v, vf, sv, svf, s), "permute sell");
  }
  check(hipStreamSynchronize(s), "sell sync");
  S.coff = coff;
  S.clen = clen;
  S.sci = sci;
  S.sv = sv;
  S.svf = svf;
  h->has_sel[which] = S.nchunks > 0;
}

// Workgroups of the SELL-64 launch for workgroup configuration cfg: two per
// CU with the 64 KB LDS slice at 1024 threads, four at 512 threads (two
// resident), sixteen per CU without it, and no more than the chunks need.
static int sell_grid(const pdlp_handle* h, int cfg, int nchunks) {
  const int cus = std::max(1, h->persist_grid / 8);
  const int waves = cfg == 0 ? 16 : (cfg == 1 ? 8 : 4);
  const int cap = cus * (cfg == 0 ? 2 : (cfg == 1 ? 4 : 16));
  return std::max(1, std::min(cap, (nchunks + waves - 1) / waves));
}

// Device copy of a column-panel layout; the matrix keeps layout 0 until chosen.
static void upload_panels(pdlp_handle* h, int which, DevCsr& M, const HostPanels& H, int64_t nnz,
                          const int32_t* ci, const double* v, const float* vf) {
  hipStream_t s = h->stream;
  const hipMemcpyKind kind = hipMemcpyHostToDevice;
  PanelCsr& S = M.pan;
  S.nseg = (int32_t)H.slot_seg.size();
  S.nsblocks = (int32_t)H.sblocks.size();
  int32_t* seg_ptr = h->dalloc<int32_t>(H.seg_ptr.size());
  int32_t* slot_seg = h->dalloc<int32_t>(H.slot_seg.size());
  int32_t* row_seg = h->dalloc<int32_t>(H.row_seg.size());
  RowBlock* sb = h->dalloc<RowBlock>(H.sblocks.size());
  int32_t* perm = h->dalloc<int32_t>((size_t)nnz);
  int32_t* pci = h->dalloc<int32_t>((size_t)nnz);
  double* pv = h->dalloc<double>((size_t)nnz);
  float* pvf = vf ? h->dalloc<float>((size_t)nnz) : nullptr;
  check(hipMemcpyAsync(seg_ptr, H.seg_ptr.data(), H.seg_ptr.size() * 4, kind, s), "upload panels");
  if (!H.slot_seg.empty())
    check(hipMemcpyAsync(slot_seg, H.slot_seg.data(), H.slot_seg.size() * 4, kind, s), "upload panels");
  check(hipMemcpyAsync(row_seg, H.row_seg.data(), H.row_seg.size() * 4, kind, s), "upload panels");
  check(hipMemcpyAsync(sb, H.sblocks.data(), H.sblocks.size() * sizeof(RowBlock), kind, s), "upload panels");
  RowBlock* sbw = h->dalloc<RowBlock>(H.sblocks_wide.size());
  check(hipMemcpyAsync(sbw, H.sblocks_wide.data(), H.sblocks_wide.size() * sizeof(RowBlock), kind, s),
        "upload panels");
  h->wide_sblocks[which] = sbw;
  h->wide_nsblocks[which] = (int32_t)H.sblocks_wide.size();
  if (nnz) check(hipMemcpyAsync(perm, H.perm.data(), (size_t)nnz * 4, kind, s), "upload panels");
  check(setup_permute(nnz, perm, ci, v, vf, pci, pv, pvf, s), "permute panels");
  check(hipStreamSynchronize(s), "panels sync");
  S.seg_ptr = seg_ptr;
  S.slot_seg = slot_seg;
  S.row_seg = row_seg;
  S.pci = pci;
  S.pv = pv;
  S.pvf = pvf;
  S.sblocks = sb;
  S.part = h->dalloc<double>(2 * (size_t)std::max(S.nseg, 1));
}

// Device copy of an LDS-staged layout for the step view of matrix `which`
// (kept in h->stg until the chooser or the option selects it).
static void upload_staged(pdlp_handle* h, int which, const HostStaged& H, const int32_t* rp, const int32_t* ci,
                          int nrows, int ncols, const int32_t* ci_dev, const double* v, const float* vf) {
  hipStream_t s = h->stream;
  const hipMemcpyKind kind = hipMemcpyHostToDevice;
  auto up = [&](const auto& vec, const char* what) {
    using T = typename std::decay_t<decltype(vec)>::value_type;
    T* d = h->dalloc<T>(vec.size());
    if (!vec.empty()) check(hipMemcpyAsync(d, vec.data(), vec.size() * sizeof(T), kind, s), what);
    return d;
  };
  StagedCsr& S = h->stg[which];
  S = StagedCsr{};
  S.nwork = (int32_t)H.wpanel.size();
  S.ncols = ncols;
  S.nseg = H.nseg;
  S.rlong = H.rlong;
  // the row pass: 64 long rows per workgroup, a thread per short row
  S.nlong_groups = std::min(kElemBlocks, (H.rlong + 63) / 64);
  S.npan = H.npan;
  S.nrblocks = std::min(kElemBlocks, (nrows - H.rlong + kBlock - 1) / kBlock);
  S.sgrid = std::max(8, ((int)H.wpanel.size() + 7) / 8 * 8);   // (a multiple of 8 already)
  S.wpanel = up(H.wpanel, "upload staged panels");
  S.wchunk = up(H.wchunk, "upload staged panels");
  S.coff = up(H.coff, "upload staged panels");
  S.clen = up(H.clen, "upload staged panels");
  S.cseg = up(H.cseg, "upload staged panels");
  S.srow = up(H.srow, "upload staged panels");
  S.pci = up(H.pci, "upload staged panels");
  const int64_t ne = std::max<int64_t>(H.nent, 1);
  int32_t* perm = h->dalloc<int32_t>((size_t)ne);
  double* pv = h->dalloc<double>((size_t)ne);
  float* pvf = vf ? h->dalloc<float>((size_t)ne) : nullptr;
  if (H.nent) {
    check(hipMemcpyAsync(perm, H.perm.data(), (size_t)H.nent * 4, kind, s), "upload staged panels");
    check(setup_permute_values(H.nent, perm, v, vf, pv, pvf, s), "permute staged panels");
  }
  S.pv = pv;
  S.pvf = pvf;
  // the dense segment sums: zero once here; a (row, panel) without nonzeros is never written
  const size_t dense = std::max<size_t>((size_t)H.npan * (size_t)H.rlong, 1);
  S.part = h->dalloc<double>(dense);
  check(hipMemsetAsync(S.part, 0, dense * sizeof(double), s), "clear staged segment sums");
  // the short rows' column panels (phase-1 blocks of kTile nonzeros)
  PanelCsr& Q = h->stg_pan[which];
  Q = PanelCsr{};
  if (H.rlong < nrows) {
    // (rows with one nonzero or none are summed directly in the row pass)
    const HostPanels HP = build_panels(rp, ci, nrows, ncols, nullptr, H.rlong, 2);
    const int64_t nz = (int64_t)HP.perm.size();
    Q.nseg = (int32_t)HP.slot_seg.size();
    Q.nsblocks = (int32_t)HP.sblocks.size();
    Q.seg_ptr = up(HP.seg_ptr, "upload short-row panels");
    Q.slot_seg = up(HP.slot_seg, "upload short-row panels");
    Q.row_seg = up(HP.row_seg, "upload short-row panels");
    Q.sblocks = up(HP.sblocks, "upload short-row panels");
    int32_t* qperm = up(HP.perm, "upload short-row panels");
    int32_t* qci = h->dalloc<int32_t>((size_t)std::max<int64_t>(nz, 1));
    double* qv = h->dalloc<double>((size_t)std::max<int64_t>(nz, 1));
    float* qvf = vf ? h->dalloc<float>((size_t)std::max<int64_t>(nz, 1)) : nullptr;
    check(setup_permute(nz, qperm, ci_dev, v, vf, qci, qv, qvf, s), "permute short-row panels");
    Q.pci = qci;
    Q.pv = qv;
    Q.pvf = qvf;
    Q.part = h->dalloc<double>((size_t)std::max(Q.nseg, 1));
  }
  check(hipStreamSynchronize(s), "staged panels sync");
  h->has_stg[which] = H.nseg > 0;
}

// The staged layout keeps its segment sums dense (panels x long rows); it
// is built only where most (long row, panel) pairs hold nonzeros, as on
// power-law LPs whose few long rows span every panel.
static bool staged_dense_ok(const HostStaged& H) {
  return (int64_t)H.npan * H.rlong <= 4 * (int64_t)H.nseg + (1 << 20);
}

// Mean duration (ms) of the step pass over K (which = 0, the dual step) or K'
// (1, the primal step) in the current layout, on a private state: current
// buffer 0, a tiny step, a pending weight of 0.  The passes then read the
// zero start buffers and write only the next-iterate buffers, dx, the
// partials and +0 into the running sums, all of which the first step of a
// solve overwrites before reading them.
static double time_probe(pdlp_handle* h, int which, int reps) {
  hipStream_t s = h->stream;
  Params T = h->P;
  T.st = h->probe_st;
  T.tr = Trace{};
  auto pass = [&]() {
    if (which) launch_primal(T, s);
    else launch_dual(T, s);
  };
  hipEvent_t a, b;
  check(hipEventCreate(&a), "hipEventCreate");
  check(hipEventCreate(&b), "hipEventCreate");
  pass();
  check(hipEventRecord(a, s), "event");
  for (int i = 0; i < reps; ++i) pass();
  check(hipEventRecord(b, s), "event");
  check(hipEventSynchronize(b), "event sync");
  float ms = 0.f;
  check(hipEventElapsedTime(&ms, a, b), "elapsed");
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms / reps;
}

// Layout of each matrix: the option's, or (spmv_layout = -1) the fastest of
// row blocks, row blocks with XCD-contiguous ranges, and column panels (when
// built), each with one workgroup per block or a persistent grid, and for the
// step passes each with kTile or kTileWide nonzeros per block, timed on the
// step passes themselves.  A candidate replaces the best so far only when
// faster by more than 2 %, and plain row blocks of kTile only when faster by
// more than 5 %, so close calls keep the earlier choice (timings move a few
// percent from run to run; the choice changes the order of sums).  The
// evaluation passes take the chosen layout with kTile blocks.
static void choose_layouts(pdlp_handle* h) {
  Params& P = h->P;
  {
    DevState z;
    std::memset(&z, 0, sizeof z);
    z.eta = 1e-6;
    z.omega = 1.0;
    z.has_pending = 1;
    h->probe_st = h->dalloc<DevState>(1);
    check(hipMemcpyAsync(h->probe_st, &z, sizeof z, hipMemcpyHostToDevice, h->stream), "probe state");
  }
  // the primal pass first: the dual pass gathers its dx
  for (int which = 1; which >= 0; --which) {
    DevCsr& M = which ? P.KT : P.K;     // the evaluation passes' view
    DevCsr& V = which ? P.KTs : P.Ks;   // the step passes' view
    const int mode = (which == 1 && h->opt.spmv_layout_kt != -2) ? h->opt.spmv_layout_kt : h->opt.spmv_layout;
    const bool has_pan = M.pan.seg_ptr != nullptr;
    // persistent grid: at most CUs x 8 workgroups (a multiple of 8, keeping
    // each workgroup on one XCD), each taking about four blocks or more
    auto pgrid = [&](int nb) {
      const int want = ((nb + 3) / 4 + 7) / 8 * 8;
      return std::max(8, std::min(h->persist_grid, want));
    };
    auto set = [&](int layout, int remap, int grid, int tile) {
      M.layout = layout;
      M.remap = remap;
      M.grid = grid ? pgrid(layout == 1 ? M.pan.nsblocks : M.nblocks) : 0;
      M.nred = layout == 1 ? M.rows_grid : M.nblocks;
      V = M;
      if (tile == kTileWide) {
        V.tile = kTileWide;
        V.blocks = h->wide_blocks[which];
        V.nblocks = h->wide_nblocks[which];
        if (layout == 1) {
          V.pan.sblocks = h->wide_sblocks[which];
          V.pan.nsblocks = h->wide_nsblocks[which];
        }
        V.grid = grid ? pgrid(layout == 1 ? V.pan.nsblocks : V.nblocks) : 0;
        V.nred = layout == 1 ? V.rows_grid : V.nblocks;
      }
    };
    // the step view in the LDS-staged layout (phase-1 workgroup size `cfg`);
    // the evaluation view then always takes column panels (else row blocks) on
    // a persistent grid, so that the layout code names the whole configuration
    auto set_staged = [&](int cfg) {
      set(has_pan ? 1 : 0, 0, 1, kTile);
      V = M;
      V.layout = 3;
      V.tile = kTile;
      V.remap = 0;
      V.grid = 0;
      V.stg = h->stg[which];
      V.stg.cfg = cfg;
      V.pan = h->stg_pan[which];
      V.nred = V.stg.nlong_groups + V.stg.nrblocks;
    };
    // both views in the SELL-64 layout (workgroup configuration `cfg`)
    auto set_sell = [&](int cfg) {
      set(0, 0, 0, kTile);
      M.layout = 4;
      M.remap = 0;
      M.grid = 0;
      M.sel = h->sel[which];
      M.sel.cfg = cfg;
      M.sel.grid = sell_grid(h, cfg, M.sel.nchunks);
      M.nred = M.sel.grid;
      V = M;
    };
    if (mode >= 0) {   // forced: bits 0-1 the layout, bit 2 the persistent grid, bit 3 the wide step tiles;
                       // 3 + 16 cfg: staged step view, column panels (else row blocks) on a persistent grid
                       // for the evaluations; 64 + 16 cfg: SELL-64 for the step and evaluation passes
      const int g = (mode & 4) ? 1 : 0, t = (mode & 8) ? kTileWide : kTile;
      if (mode & 64) {
        if (h->has_sel[which]) set_sell((mode >> 4) & 3);
        else set(has_pan ? 1 : 0, 0, 1, kTile);
      } else if ((mode & 3) == 0) set(0, 0, g, t);
      else if ((mode & 3) == 2) set(0, 1, g, t);
      else if ((mode & 3) == 1) set(has_pan ? 1 : 0, 0, g, t);
      else if (h->has_stg[which]) set_staged((mode >> 4) & 3);
      else set(has_pan ? 1 : 0, 0, 1, kTile);
      continue;
    }
    set(0, 0, 0, kTile);
    if (h->nnz < (1 << 20)) continue;   // small problems: row blocks
    const double base = time_probe(h, which, 6);
    double best = INFINITY;
    int best_l = 0, best_r = 0, best_g = 0, best_t = kTile;
    const int cands[3][2] = {{0, 0}, {0, 1}, {1, 0}};
    for (int tile : {kTile, kTileWide}) {
      for (const auto& c : cands) {
        if (c[0] == 1 && !has_pan) continue;
        for (int g : {0, 1}) {
          if (tile == kTile && c[0] == 0 && c[1] == 0 && g == 0) continue;   // the baseline, timed above
          set(c[0], c[1], g, tile);
          const double t = time_probe(h, which, 6);
          if (t < 0.98 * best) {
            best = t;
            best_l = c[0];
            best_r = c[1];
            best_g = g;
            best_t = tile;
          }
        }
      }
    }
    if (!(best < 0.95 * base)) {
      best = base;
      best_l = best_r = best_g = 0;
      best_t = kTile;
    }
    set(best_l, best_r, best_g, best_t);
    if (h->has_stg[which]) {
      int best_c = -1;
      for (int cfg = 0; cfg < 3; ++cfg) {
        set_staged(cfg);
        const double t = time_probe(h, which, 6);
        if (t < 0.98 * best) {
          best = t;
          best_c = cfg;
        }
      }
      set(best_l, best_r, best_g, best_t);
      if (best_c >= 0) set_staged(best_c);
    }
    if (h->has_sel[which]) {
      // (the current view is the best so far; keep a copy to come back to)
      const DevCsr bm = M, bv = V;
      int best_c = -1;
      for (int cfg = 0; cfg < 3; ++cfg) {
        set_sell(cfg);
        const double t = time_probe(h, which, 6);
        if (t < 0.98 * best) {
          best = t;
          best_c = cfg;
        }
      }
      M = bm;
      V = bv;
      if (best_c >= 0) set_sell(best_c);
    }
    h->probe_ms[which] = best;
  }
}

static int load_problem(const pdlp_problem* p, void* hip_stream, HostLP& H, std::string& why) {
  if (p->m < 0 || p->n < 1 || p->nnz < 0 || p->nnz >= (int64_t)1 << 31)
    return why = "sizes must satisfy m >= 0, n >= 1, 0 <= nnz < 2^31", PDLP_ERR_ARG;
  if (p->mem != PDLP_MEM_HOST && p->mem != PDLP_MEM_DEVICE) return why = "bad mem kind", PDLP_ERR_ARG;
  if (!p->row_ptr || !p->c || !p->l || !p->u || (p->nnz > 0 && (!p->col_idx || !p->val)) ||
      (p->m > 0 && (!p->b || !p->row_type)))
    return why = "NULL problem array", PDLP_ERR_ARG;
  H.m = p->m;
  H.n = p->n;
  H.nnz = p->nnz;
  try {
    if (p->mem == PDLP_MEM_DEVICE) {
      int ndev = 0;
      check(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
      // the caller's producers of the device arrays run on its stream
      check(hipStreamSynchronize((hipStream_t)hip_stream), "hipStreamSynchronize");
    }
    fetch(H.rp, p->row_ptr, (size_t)H.m + 1, p->mem);
    fetch(H.ci, p->col_idx, (size_t)H.nnz, p->mem);
    fetch(H.v, p->val, (size_t)H.nnz, p->mem);
    fetch(H.c, p->c, (size_t)H.n, p->mem);
    fetch(H.b, p->b, (size_t)H.m, p->mem);
    fetch(H.l, p->l, (size_t)H.n, p->mem);
    fetch(H.u, p->u, (size_t)H.n, p->mem);
    fetch(H.rt, p->row_type, (size_t)H.m, p->mem);
  } catch (const HipFail& f) {
    return why = hip_msg(f), PDLP_ERR_HIP;
  }
  if (validate(H.m, H.n, H.nnz, H.rp.data(), H.ci.data(), H.v.data(), H.c.data(), H.b.data(), H.l.data(),
               H.u.data(), H.rt.data(), why))
    return PDLP_ERR_DATA;
  return PDLP_OK;
}

// Pack LPs block-diagonally on the host, each one validated on its own (the
// message names the first bad LP).
int pdlp::pack_problems(const pdlp_problem* ps, int32_t count, void* hip_stream, HostLP& H,
                        std::vector<int32_t>& row_off, std::vector<int32_t>& col_off, std::vector<int64_t>& nnz_b,
                        std::string& why) {
  row_off.assign(1, 0);
  col_off.assign(1, 0);
  nnz_b.clear();
  int64_t M = 0, N = 0, NZ = 0;
  H = HostLP{};
  H.rp.push_back(0);
  for (int32_t k = 0; k < count; ++k) {
    HostLP L;
    if (int rc = load_problem(&ps[k], hip_stream, L, why)) {
      why = "LP " + std::to_string(k) + ": " + why;
      return rc;
    }
    if (M + L.m >= ((int64_t)1 << 31) || N + L.n >= ((int64_t)1 << 31) || NZ + L.nnz >= ((int64_t)1 << 31)) {
      why = "the packed LPs need total rows, columns and nonzeros below 2^31";
      return PDLP_ERR_ARG;
    }
    for (int32_t r = 0; r < L.m; ++r) H.rp.push_back((int32_t)(NZ + L.rp[(size_t)r + 1]));
    for (int64_t e = 0; e < L.nnz; ++e) H.ci.push_back((int32_t)(N + L.ci[(size_t)e]));
    H.v.insert(H.v.end(), L.v.begin(), L.v.begin() + L.nnz);
    H.c.insert(H.c.end(), L.c.begin(), L.c.begin() + L.n);
    H.l.insert(H.l.end(), L.l.begin(), L.l.begin() + L.n);
    H.u.insert(H.u.end(), L.u.begin(), L.u.begin() + L.n);
    H.b.insert(H.b.end(), L.b.begin(), L.b.begin() + L.m);
    H.rt.insert(H.rt.end(), L.rt.begin(), L.rt.begin() + L.m);
    M += L.m;
    N += L.n;
    NZ += L.nnz;
    row_off.push_back((int32_t)M);
    col_off.push_back((int32_t)N);
    nnz_b.push_back(L.nnz);
  }
  H.m = (int32_t)M;
  H.n = (int32_t)N;
  H.nnz = NZ;
  for (auto* vec : {&H.v, &H.c, &H.l, &H.u, &H.b}) if (vec->empty()) vec->push_back(0.0);
  if (H.ci.empty()) H.ci.push_back(0);
  if (H.rt.empty()) H.rt.push_back(0);
  return PDLP_OK;
}

// a1-a2: upload the LP, negate LE rows into the >= form, transpose on the device.
static void upload_normalize_transpose(pdlp_handle* h, const HostLP& H) {
  const int32_t m = H.m, n = H.n;
  const int64_t nnz = H.nnz;
  hipStream_t s = h->stream;
  h->rp = h->dalloc<int32_t>((size_t)m + 1);
  h->ci = h->dalloc<int32_t>((size_t)nnz);
  h->val = h->dalloc<double>((size_t)nnz);
  h->c0 = h->dalloc<double>(n);
  h->l0 = h->dalloc<double>(n);
  h->u0 = h->dalloc<double>(n);
  h->b0 = h->dalloc<double>(m);
  h->rt = h->dalloc<int8_t>(m);
  const hipMemcpyKind kind = hipMemcpyHostToDevice;
  check(hipMemcpyAsync(h->rp, H.rp.data(), ((size_t)m + 1) * 4, kind, s), "upload row_ptr");
  if (nnz) check(hipMemcpyAsync(h->ci, H.ci.data(), (size_t)nnz * 4, kind, s), "upload col_idx");
  if (nnz) check(hipMemcpyAsync(h->val, H.v.data(), (size_t)nnz * 8, kind, s), "upload val");
  check(hipMemcpyAsync(h->c0, H.c.data(), (size_t)n * 8, kind, s), "upload c");
  check(hipMemcpyAsync(h->l0, H.l.data(), (size_t)n * 8, kind, s), "upload l");
  check(hipMemcpyAsync(h->u0, H.u.data(), (size_t)n * 8, kind, s), "upload u");
  if (m) check(hipMemcpyAsync(h->b0, H.b.data(), (size_t)m * 8, kind, s), "upload b");
  if (m) check(hipMemcpyAsync(h->rt, H.rt.data(), (size_t)m, kind, s), "upload row_type");
  h->q = h->dalloc<double>(m);
  h->ineq = h->dalloc<int8_t>(m);
  h->le = h->dalloc<int8_t>(m);
  h->rowid = h->dalloc<int32_t>((size_t)nnz);
  check(setup_normalize(m, h->rp, h->val, h->b0, h->rt, h->q, h->ineq, h->le, h->rowid, s), "normalize");
  h->rpT = h->dalloc<int32_t>((size_t)n + 1);
  h->ciT = h->dalloc<int32_t>((size_t)nnz);
  h->valT = h->dalloc<double>((size_t)nnz);
  h->rowidT = h->dalloc<int32_t>((size_t)nnz);
  h->perm = h->dalloc<int32_t>((size_t)nnz);
  check(setup_transpose(m, n, nnz, h->ci, h->val, h->rowid, h->rpT, h->ciT, h->valT, h->rowidT, h->perm, s),
        "transpose");
}

// a3: Ruiz and Pock-Chambolle preconditioning (Section 2.2), then the scaled
// vectors c~, l~, u~, q~ and (FP32 steps) the rounded matrix copies.
static void scale_problem(pdlp_handle* h) {
  const int32_t m = h->m, n = h->n;
  const int64_t nnz = h->nnz;
  hipStream_t s = h->stream;
  h->D1 = h->dalloc<double>(m);
  h->D2 = h->dalloc<double>(n);
  double* d1 = h->dalloc<double>(m);
  double* d2 = h->dalloc<double>(n);
  check(setup_fill(m, h->D1, 1.0, s), "fill D1");
  check(setup_fill(n, h->D2, 1.0, s), "fill D2");
  check(setup_scale(m, n, nnz, h->rp, h->ci, h->rowid, h->val, h->rpT, h->ciT, h->rowidT, h->valT,
                    h->opt.ruiz_iters, h->opt.pc_alpha, h->D1, h->D2, d1, d2, s),
        "scale");
  h->c = h->dalloc<double>(n);
  h->l = h->dalloc<double>(n);
  h->u = h->dalloc<double>(n);
  check(setup_vectors(m, n, h->D1, h->D2, h->c0, h->l0, h->u0, h->c, h->l, h->u, h->q, s), "scale vectors");
  if (h->opt.a_precision == PDLP_A_FP32) {
    h->valf = h->dalloc<float>((size_t)nnz);
    h->valTf = h->dalloc<float>((size_t)nnz);
    check(setup_to_f32(nnz, h->val, h->valf, s), "fp32 K");
    check(setup_to_f32(nnz, h->valT, h->valTf, s), "fp32 K'");
  }
}

// Column renumbering (row_order = 2, or 1 on LPs with 2^20 nonzeros or more,
// unless the given order already fills 64-column chunks with at most 1/8
// padding): the columns sorted by descending number of nonzeros (equal
// counts in the given order) are cut into groups of 64, and the groups are dealt out over
// the column range in kStageWidth-wide strides (group i of G goes to the
// (i mod P)-th run, P = the number of kStageWidth-column panels).  Each run
// of 64 columns then has (nearly) equal counts -- the SELL-64 chunks of K~'
// need little padding -- while every wide column range still holds columns
// of every count, as in the given order, so column panels keep balanced
// entry counts.  Done after the scaling and before the row renumbering: K~'s
// entries keep their place with new column indices, the rows of K~' move
// whole, and c, l, u and D2 follow.  H.ci gets the new indices.
static void renumber_cols(pdlp_handle* h, HostLP& H) {
  const int32_t n = h->n;
  const int64_t nnz = h->nnz;
  const int ro = h->opt.row_order;
  if (!(ro == 2 || (ro == 1 && nnz >= (1 << 20))) || n < 2) return;
  std::vector<int32_t> cnt((size_t)n, 0);
  for (int64_t e = 0; e < nnz; ++e) cnt[(size_t)H.ci[(size_t)e]]++;
  {
    // the given order already fills 64-column chunks with at most 1/8
    // padding (e.g. equal counts): keep it
    int64_t padded = 0;
    for (int32_t j0 = 0; j0 < n; j0 += 64) {
      int32_t mx = 0;
      for (int32_t j = j0; j < std::min(n, j0 + 64); ++j) mx = std::max(mx, cnt[(size_t)j]);
      padded += (int64_t)64 * mx;
    }
    if (padded * 8 <= nnz * 9) return;
  }
  std::vector<int32_t> perm((size_t)n);
  for (int32_t j = 0; j < n; ++j) perm[(size_t)j] = j;
  std::stable_sort(perm.begin(), perm.end(),
                   [&](int32_t a, int32_t b) { return cnt[(size_t)a] > cnt[(size_t)b]; });
  {
    // full groups of 64 dealt out over the panels; a last partial group stays last
    const int32_t G = n / 64, P = std::max(1, (n + kStageWidth - 1) / kStageWidth);
    std::vector<int32_t> dealt;
    dealt.reserve((size_t)n);
    for (int32_t r = 0; r < P; ++r)
      for (int32_t i = r; i < G; i += P)
        for (int l = 0; l < 64; ++l) dealt.push_back(perm[(size_t)i * 64 + l]);
    for (int32_t j = G * 64; j < n; ++j) dealt.push_back(perm[(size_t)j]);
    perm.swap(dealt);
  }
  bool ident = true;
  for (int32_t j = 0; j < n && ident; ++j) ident = perm[(size_t)j] == j;
  if (ident) return;
  std::vector<int32_t> inv((size_t)n);
  for (int32_t j = 0; j < n; ++j) inv[(size_t)perm[(size_t)j]] = j;
  hipStream_t s = h->stream;
  std::vector<int32_t> rpT((size_t)n + 1), rpT2((size_t)n + 1, 0), src((size_t)std::max<int64_t>(nnz, 1));
  check(hipMemcpy(rpT.data(), h->rpT, ((size_t)n + 1) * 4, hipMemcpyDeviceToHost), "read rowptr of K'");
  for (int32_t j = 0; j < n; ++j) {
    const int32_t o = perm[(size_t)j], b = rpT[(size_t)o], L = rpT[(size_t)o + 1] - b;
    rpT2[(size_t)j + 1] = rpT2[(size_t)j] + L;
    for (int32_t k = 0; k < L; ++k) src[(size_t)rpT2[(size_t)j] + k] = b + k;
  }
  const hipMemcpyKind kind = hipMemcpyHostToDevice, d2d = hipMemcpyDeviceToDevice;
  // scratch of the move, freed before returning
  std::vector<void*> tmp;
  auto talloc = [&](size_t bytes) {
    void* p = nullptr;
    check(hipMalloc(&p, std::max<size_t>(bytes, 1)), "hipMalloc");
    tmp.push_back(p);
    return p;
  };
  try {
    int32_t* d_src = static_cast<int32_t*>(talloc((size_t)nnz * 4));
    int32_t* d_perm = static_cast<int32_t*>(talloc((size_t)n * 4));
    int32_t* d_inv = static_cast<int32_t*>(talloc((size_t)n * 4));
    int32_t* t_ci = static_cast<int32_t*>(talloc((size_t)nnz * 4));
    double* t_v = static_cast<double*>(talloc((size_t)nnz * 8));
    float* t_vf = h->valTf ? static_cast<float*>(talloc((size_t)nnz * 4)) : nullptr;
    double* t_col = static_cast<double*>(talloc((size_t)n * 8));
    if (nnz) check(hipMemcpyAsync(d_src, src.data(), (size_t)nnz * 4, kind, s), "upload renumbering");
    check(hipMemcpyAsync(d_perm, perm.data(), (size_t)n * 4, kind, s), "upload renumbering");
    check(hipMemcpyAsync(d_inv, inv.data(), (size_t)n * 4, kind, s), "upload renumbering");
    // K~': rows moved whole
    check(setup_permute(nnz, d_src, h->ciT, h->valT, h->valTf, t_ci, t_v, t_vf, s), "renumber K'");
    if (nnz) {
      check(hipMemcpyAsync(h->ciT, t_ci, (size_t)nnz * 4, d2d, s), "renumber K'");
      check(hipMemcpyAsync(h->valT, t_v, (size_t)nnz * 8, d2d, s), "renumber K'");
      if (h->valTf) check(hipMemcpyAsync(h->valTf, t_vf, (size_t)nnz * 4, d2d, s), "renumber K'");
    }
    check(hipMemcpyAsync(h->rpT, rpT2.data(), ((size_t)n + 1) * 4, kind, s), "renumber K'");
    // K~: new column indices in place
    check(setup_rename(nnz, d_inv, h->ci, s), "renumber K");
    // column vectors
    for (double* v : {h->c, h->l, h->u, h->D2}) {
      check(setup_gather_rows(n, d_perm, v, t_col, s), "renumber columns");
      check(hipMemcpyAsync(v, t_col, (size_t)n * 8, d2d, s), "renumber columns");
    }
    check(hipStreamSynchronize(s), "renumber sync");
  } catch (const HipFail&) {
    for (void* p : tmp) (void)hipFree(p);
    throw;
  }
  for (void* p : tmp) (void)hipFree(p);
  for (int64_t e = 0; e < nnz; ++e) H.ci[(size_t)e] = inv[(size_t)H.ci[(size_t)e]];
  h->cperm = std::move(perm);
}

// Row renumbering for the locality of the gathers: rows by descending length,
// equal lengths by their first column, then by index.  On a power-law LP the
// few long rows that hold most nonzeros get the first entries of y (the
// primal step's gathers of y then stay in L1 and L2), and the many short rows
// follow their columns (gathers in increasing address order).  Done after the
// scaling, so D1, D2 and K~ are those of the given order: K~'s entries keep
// their place (each column is summed in the same order) with new row indices,
// and K~'s rows move whole.  H.rp and H.ci become the new structure.
static void renumber_rows(pdlp_handle* h, HostLP& H) {
  const int32_t m = h->m;
  const int64_t nnz = h->nnz;
  if (!h->opt.row_order || m < 2) return;
  std::vector<int32_t> perm((size_t)m);
  for (int32_t r = 0; r < m; ++r) perm[(size_t)r] = r;
  auto len = [&](int32_t r) { return H.rp[(size_t)r + 1] - H.rp[(size_t)r]; };
  auto first = [&](int32_t r) { return len(r) > 0 ? H.ci[(size_t)H.rp[(size_t)r]] : INT32_MAX; };
  std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) {
    const int32_t la = len(a), lb = len(b);
    if (la != lb) return la > lb;
    return first(a) < first(b);
  });
  bool ident = true;
  for (int32_t r = 0; r < m && ident; ++r) ident = perm[(size_t)r] == r;
  if (ident) return;
  std::vector<int32_t> rp2((size_t)m + 1, 0), src((size_t)std::max<int64_t>(nnz, 1)), inv((size_t)m);
  std::vector<int32_t> ci2((size_t)std::max<int64_t>(nnz, 1));
  for (int32_t r = 0; r < m; ++r) {
    const int32_t o = perm[(size_t)r], b = H.rp[(size_t)o], L = len(o);
    rp2[(size_t)r + 1] = rp2[(size_t)r] + L;
    for (int32_t k = 0; k < L; ++k) {
      src[(size_t)rp2[(size_t)r] + k] = b + k;
      ci2[(size_t)rp2[(size_t)r] + k] = H.ci[(size_t)b + k];
    }
    inv[(size_t)o] = r;
  }
  hipStream_t s = h->stream;
  const hipMemcpyKind kind = hipMemcpyHostToDevice;
  // scratch of the move, freed before returning
  std::vector<void*> tmp;
  auto talloc = [&](size_t bytes) {
    void* p = nullptr;
    check(hipMalloc(&p, std::max<size_t>(bytes, 1)), "hipMalloc");
    tmp.push_back(p);
    return p;
  };
  try {
    int32_t* d_src = static_cast<int32_t*>(talloc((size_t)nnz * 4));
    int32_t* d_perm = static_cast<int32_t*>(talloc((size_t)m * 4));
    int32_t* d_inv = static_cast<int32_t*>(talloc((size_t)m * 4));
    int32_t* t_ci = static_cast<int32_t*>(talloc((size_t)nnz * 4));
    double* t_v = static_cast<double*>(talloc((size_t)nnz * 8));
    float* t_vf = h->valf ? static_cast<float*>(talloc((size_t)nnz * 4)) : nullptr;
    double* t_row = static_cast<double*>(talloc((size_t)m * 8));
    int8_t* t_row8 = static_cast<int8_t*>(talloc((size_t)m));
    if (nnz) check(hipMemcpyAsync(d_src, src.data(), (size_t)nnz * 4, kind, s), "upload renumbering");
    check(hipMemcpyAsync(d_perm, perm.data(), (size_t)m * 4, kind, s), "upload renumbering");
    check(hipMemcpyAsync(d_inv, inv.data(), (size_t)m * 4, kind, s), "upload renumbering");
    // K~: rows moved whole
    check(setup_permute(nnz, d_src, h->ci, h->val, h->valf, t_ci, t_v, t_vf, s), "renumber K");
    const hipMemcpyKind d2d = hipMemcpyDeviceToDevice;
    if (nnz) {
      check(hipMemcpyAsync(h->ci, t_ci, (size_t)nnz * 4, d2d, s), "renumber K");
      check(hipMemcpyAsync(h->val, t_v, (size_t)nnz * 8, d2d, s), "renumber K");
      if (h->valf) check(hipMemcpyAsync(h->valf, t_vf, (size_t)nnz * 4, d2d, s), "renumber K");
    }
    check(hipMemcpyAsync(h->rp, rp2.data(), ((size_t)m + 1) * 4, kind, s), "renumber K");
    // K~': new row indices in place
    check(setup_rename(nnz, d_inv, h->ciT, s), "renumber K'");
    // row vectors
    for (double* v : {h->q, h->D1, h->b0}) {
      check(setup_gather_rows(m, d_perm, v, t_row, s), "renumber rows");
      check(hipMemcpyAsync(v, t_row, (size_t)m * 8, d2d, s), "renumber rows");
    }
    for (int8_t* v : {h->ineq, h->le, h->rt}) {
      check(setup_gather_rows_i8(m, d_perm, v, t_row8, s), "renumber rows");
      check(hipMemcpyAsync(v, t_row8, (size_t)m, d2d, s), "renumber rows");
    }
    check(hipStreamSynchronize(s), "renumber sync");
  } catch (const HipFail&) {
    for (void* p : tmp) (void)hipFree(p);
    throw;
  }
  for (void* p : tmp) (void)hipFree(p);
  h->rp_given = H.rp;
  h->rp_dev = rp2;
  h->rperm = std::move(perm);
  H.rp = std::move(rp2);
  H.ci = std::move(ci2);
}

// Iterate, average and output buffers and the constants of Params.
static void alloc_iterates(pdlp_handle* h) {
  const int32_t m = h->m, n = h->n;
  const pdlp_options& opt = h->opt;
  Params& P = h->P;
  P.m = m;
  P.n = n;
  P.use_f32 = opt.a_precision == PDLP_A_FP32;
  for (int k = 0; k < 2; ++k) {
    P.x[k] = h->dalloc<double>(n);
    P.y[k] = h->dalloc<double>(m);
    P.kx[k] = h->dalloc<double>(m);
  }
  P.dx = h->dalloc<double>(n);
  P.xsum = h->dalloc<double>(n);
  P.ysum = h->dalloc<double>(m);
  P.xbar = h->dalloc<double>(n);
  P.ybar = h->dalloc<double>(m);
  P.x0 = h->dalloc<double>(n);
  P.y0 = h->dalloc<double>(m);
  P.c = h->c;
  P.q = h->q;
  P.l = h->l;
  P.u = h->u;
  P.ineq = h->ineq;
  P.le = h->le;
  P.D1 = h->D1;
  P.D2 = h->D2;
  if (opt.trace > 0) {
    const size_t cap = (size_t)opt.trace;
    P.tr = Trace{(int64_t)cap,
                 h->dalloc<int64_t>(cap), h->dalloc<double>(cap), h->dalloc<double>(cap), h->dalloc<int8_t>(cap),
                 h->dalloc<int64_t>(cap), h->dalloc<double>(cap), h->dalloc<double>(cap), h->dalloc<int8_t>(cap),
                 h->dalloc<int8_t>(cap), h->dalloc<double>(cap)};
  } else {
    P.tr = Trace{};
  }
  P.P = opt.eval_period;
  P.beta_suff = opt.beta_suff;
  P.beta_nec = opt.beta_nec;
  P.beta_art = opt.beta_art;
  P.theta = opt.pw_theta;
  P.eps_zero = opt.eps_zero;
  P.tie_rel = 1e-12;
  P.omega_power = opt.kkt_omega_power;
  P.infeas = opt.detect_infeas;
  P.eps_infeas = opt.eps_infeas;
  P.infeas_every = opt.infeas_every;
  P.gap = opt.restart_metric == 1;
  if (P.gap) {
    for (int k = 0; k < 2; ++k) {
      P.kxe[k] = h->dalloc<double>(m);
      P.ktye[k] = h->dalloc<double>(n);
    }
    P.partG = h->dalloc<double>((size_t)kGapAcc * 2 * kElemBlocks);
  }
  if (P.infeas) {
    for (int k = 0; k < 2; ++k) {
      P.xr[k] = h->dalloc<double>(n);
      P.yr[k] = h->dalloc<double>(m);
    }
  }
  h->xo = h->dalloc<double>(n);
  h->yo = h->dalloc<double>(m);
  h->rco = h->dalloc<double>(n);
  P.xo = h->xo;
  P.yo = h->yo;
  P.rco = h->rco;
  h->wx = h->dalloc<double>(n);
  h->wy = h->dalloc<double>(m);
}

static int create_failed(pdlp_handle* h, const HipFail& f) {
  std::string msg = hip_msg(f);
  const int code = (f.e == hipErrorOutOfMemory || f.e == hipErrorMemoryAllocation) ? PDLP_ERR_OOM : PDLP_ERR_HIP;
  h->release();
  delete h;
  return fail(nullptr, code, msg);
}

extern "C" int pdlp_create(const pdlp_problem* p, const pdlp_options* o, void* hip_stream, pdlp_handle** out) {
  if (out) *out = nullptr;
  if (!p || !out) return fail(nullptr, PDLP_ERR_ARG, "NULL problem or output pointer");
  pdlp_options opt;
  if (o) opt = *o;
  else pdlp_default_options(&opt);
  std::string why;
  if (check_options(opt, why)) return fail(nullptr, PDLP_ERR_ARG, why);
  const double t0 = now_s();
  HostLP H;
  if (int rc = load_problem(p, hip_stream, H, why)) return fail(nullptr, rc, why);
  Presolve pre;
  HostLP orig;
  bool presolved = false;
  if (opt.presolve) {
    // the reduced LP replaces the user's; an LP that presolve finds infeasible,
    // or reduces to no column, is solved as given (the method then returns
    // its certificate, or the postsolve would have nothing to run)
    HostLP R;
    if (presolve_lp(H, R, pre) == 0 && R.n >= 1) {
      orig = std::move(H);
      H = std::move(R);
      presolved = true;
    }
  }
  const int32_t m = H.m, n = H.n;
  const int64_t nnz = H.nnz;

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(nullptr, PDLP_ERR_HIP, "no HIP device");

  pdlp_handle* h = new pdlp_handle();
  h->m = m;
  h->n = n;
  h->nnz = nnz;
  h->opt = opt;
  h->stream = (hipStream_t)hip_stream;
  h->presolved = presolved;
  if (presolved) {
    h->pre = std::move(pre);
    h->orig = std::move(orig);
  }
  try {
    check(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
    {
      hipDeviceProp_t prop;
      int dev = 0;
      check(hipGetDevice(&dev), "hipGetDevice");
      check(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
      h->persist_grid = std::max(8, prop.multiProcessorCount * 8);
      h->device = dev;
    }
    hipStream_t s = h->stream;
    const hipMemcpyKind kind = hipMemcpyHostToDevice;
    upload_normalize_transpose(h, H);
    // unscaled norms of the Section 4.1 tests
    double* red = h->dalloc<double>(8);
    double* part = h->dalloc<double>((size_t)std::max<int64_t>(n, m) / 4096 + 2);
    check(setup_sumsq(n, h->c0, part, red + 0, s), "norm c");
    check(setup_sumsq(m, h->q, part, red + 1, s), "norm q");
    scale_problem(h);
    // --- a4: omega0 = ||c~|| / ||q~||, eta0 = 1 / max |K~|
    check(setup_sumsq(n, h->c, part, red + 2, s), "norm c~");
    check(setup_sumsq(m, h->q, part, red + 3, s), "norm q~");
    check(setup_absmax(nnz, h->val, reinterpret_cast<unsigned long long*>(red + 4), s), "max |K~|");
    double hred[5];
    check(hipMemcpyAsync(hred, red, sizeof hred, hipMemcpyDeviceToHost, s), "read norms");
    check(hipStreamSynchronize(s), "setup sync");
    const double cn = std::sqrt(hred[2]), qn = std::sqrt(hred[3]);
    h->omega0 = (cn > opt.eps_zero && qn > opt.eps_zero) ? cn / qn : 1.0;
    double kmax;
    std::memcpy(&kmax, &hred[4], sizeof kmax);
    h->eta0 = kmax > 0.0 ? 1.0 / kmax : 1.0;
    renumber_cols(h, H);
    renumber_rows(h, H);
    // --- row-block partitions and (optionally) the column-panel layouts
    std::vector<int32_t> hrpT((size_t)n + 1);
    check(hipMemcpy(hrpT.data(), h->rpT, ((size_t)n + 1) * 4, hipMemcpyDeviceToHost), "read rowptr of K'");
    std::vector<RowBlock> bk = partition_rows(H.rp.data(), m);
    std::vector<RowBlock> bt = partition_rows(hrpT.data(), n);
    RowBlock* dbk = h->dalloc<RowBlock>(bk.size());
    RowBlock* dbt = h->dalloc<RowBlock>(bt.size());
    check(hipMemcpyAsync(dbk, bk.data(), bk.size() * sizeof(RowBlock), kind, s), "upload blocks");
    check(hipMemcpyAsync(dbt, bt.data(), bt.size() * sizeof(RowBlock), kind, s), "upload blocks");
    // the wider tiling a step pass may take (chosen with the layout)
    for (int which = 0; which < 2; ++which) {
      std::vector<RowBlock> w = partition_rows(which ? hrpT.data() : H.rp.data(), 0, which ? n : m, kTileWide);
      if (w.empty()) w.push_back(RowBlock{0, 0});
      RowBlock* dw = h->dalloc<RowBlock>(w.size());
      check(hipMemcpyAsync(dw, w.data(), w.size() * sizeof(RowBlock), kind, s), "upload blocks");
      h->wide_blocks[which] = dw;
      h->wide_nblocks[which] = (int32_t)w.size();
    }
    Params& P = h->P;
    P.K = DevCsr{h->rp, h->ci, h->val, h->valf, dbk, (int32_t)bk.size(), m, 0, 0, 0, elem_grid(m), 0, PanelCsr{}};
    P.KT = DevCsr{h->rpT, h->ciT, h->valT, h->valTf, dbt, (int32_t)bt.size(), n, 0, 0, 0, elem_grid(n), 0,
                  PanelCsr{}};
    // a panel layout pays when the gathered vector does not fit one XCD's L2;
    // spmv_layout = 1 builds it for any size (tests)
    const int mode_k = opt.spmv_layout, mode_kt = opt.spmv_layout_kt != -2 ? opt.spmv_layout_kt : opt.spmv_layout;
    // (a staged or SELL code builds it under the size rule of the automatic
    // choice, so that its evaluation passes take the same layout either way)
    auto step_code = [](int mode) { return mode == -1 || (mode & 3) == 3 || mode >= 64; };
    const bool want_k = (mode_k >= 0 && mode_k < 64 && (mode_k & 3) == 1) ||
                        (step_code(mode_k) && nnz >= (1 << 20) && n >= (1 << 18));
    const bool want_kt = (mode_kt >= 0 && mode_kt < 64 && (mode_kt & 3) == 1) ||
                         (step_code(mode_kt) && nnz >= (1 << 20) && m >= (1 << 18));
    {
      std::vector<int32_t> hciT;
      if (want_k) {
        HostPanels HP = build_panels(H.rp.data(), H.ci.data(), m, n, hrpT.data());
        upload_panels(h, 0, P.K, HP, nnz, h->ci, h->val, h->valf);
      }
      if (want_kt) {
        hciT.resize((size_t)std::max<int64_t>(nnz, 1));
        if (nnz) check(hipMemcpy(hciT.data(), h->ciT, (size_t)nnz * 4, hipMemcpyDeviceToHost), "read K' columns");
        HostPanels HP = build_panels(hrpT.data(), hciT.data(), n, m, H.rp.data());
        upload_panels(h, 1, P.KT, HP, nnz, h->ciT, h->valT, h->valTf);
      }
    }
    // the LDS-staged step layouts: when the long rows (at least kStageMinLen
    // nonzeros, numbered first) hold most of the nonzeros and the gathered
    // vector is large; spmv_layout = 3 (+16 cfg) builds them for any size (tests)
    {
      const bool force_k = mode_k >= 0 && (mode_k & 3) == 3, force_kt = mode_kt >= 0 && (mode_kt & 3) == 3;
      const bool auto_k = mode_k == -1 && nnz >= (1 << 20) && n >= (1 << 18);
      const bool auto_kt = mode_kt == -1 && nnz >= (1 << 20) && m >= (1 << 18);
      if (force_k || auto_k) {
        const int64_t nl = leading_long_nnz(H.rp.data(), m, kStageMinLen);
        if (force_k || 2 * nl >= nnz) {
          HostStaged HS = build_staged(H.rp.data(), H.ci.data(), m, n, kStageMinLen, h->persist_grid / 8);
          if (staged_dense_ok(HS)) upload_staged(h, 0, HS, H.rp.data(), H.ci.data(), m, n, h->ci, h->val, h->valf);
        }
      }
      if (force_kt || auto_kt) {
        const int64_t nl = leading_long_nnz(hrpT.data(), n, kStageMinLen);
        if (force_kt || 2 * nl >= nnz) {
          std::vector<int32_t> hciT((size_t)std::max<int64_t>(nnz, 1));
          if (nnz) check(hipMemcpy(hciT.data(), h->ciT, (size_t)nnz * 4, hipMemcpyDeviceToHost), "read K' columns");
          HostStaged HS = build_staged(hrpT.data(), hciT.data(), n, m, kStageMinLen, h->persist_grid / 8);
          if (staged_dense_ok(HS))
            upload_staged(h, 1, HS, hrpT.data(), hciT.data(), n, m, h->ciT, h->valT, h->valTf);
        }
      }
    }
    // the SELL-64 step layouts: when a matrix's rows, in their device
    // numbering, fill chunks of 64 rows with at most 1/8 padding, give at
    // least four chunks per CU, and none is longer than 16 times the mean
    // (plus 64: one lane sums a whole row, so a long row would hold its
    // chunk's wavefront long after the others), under the size rule of the
    // automatic choice, or for any size when forced
    auto balanced = [&](const int32_t* rp, int nrows) {
      if ((int64_t)nrows < (int64_t)64 * 4 * std::max(1, h->persist_grid / 8)) return false;
      int32_t mx = 0;
      for (int r = 0; r < nrows; ++r) mx = std::max(mx, rp[r + 1] - rp[r]);
      return (int64_t)mx <= 16 * (nnz / std::max(nrows, 1)) + 64;
    };
    {
      const bool force_k = mode_k >= 64, force_kt = mode_kt >= 64;
      const bool auto_k = mode_k == -1 && nnz >= (1 << 20) && balanced(H.rp.data(), m);
      const bool auto_kt = mode_kt == -1 && nnz >= (1 << 20) && balanced(hrpT.data(), n);
      if (force_k || auto_k) {
        HostSell HS = build_sell(H.rp.data(), H.ci.data(), m);
        if (HS.nent >= 0 && (force_k || HS.nent * 8 <= nnz * 9)) upload_sell(h, 0, HS, n, h->val, h->valf);
      }
      if (force_kt || auto_kt) {
        std::vector<int32_t> hciT((size_t)std::max<int64_t>(nnz, 1));
        if (nnz) check(hipMemcpy(hciT.data(), h->ciT, (size_t)nnz * 4, hipMemcpyDeviceToHost), "read K' columns");
        HostSell HS = build_sell(hrpT.data(), hciT.data(), n);
        if (HS.nent >= 0 && (force_kt || HS.nent * 8 <= nnz * 9)) upload_sell(h, 1, HS, m, h->valT, h->valTf);
      }
    }
    P.Ks = P.K;
    P.KTs = P.KT;
    alloc_iterates(h);
    // K~x_bar of the evaluations' split row pass (on an FP64 LDS-staged view of K~)
    if (h->has_stg[0] && !P.use_f32) P.kxb = h->dalloc<double>((size_t)std::max(m, 1));
    // partials: one per block of either tiling, or per workgroup of the row pass
    // (and per workgroup of the staged layouts' row pass)
    auto stg_red = [&](int w) {
      return h->has_stg[w] ? (size_t)(h->stg[w].nlong_groups + h->stg[w].nrblocks) : (size_t)0;
    };
    auto sel_red = [&](int w) {
      size_t g = 0;
      if (h->has_sel[w])
        for (int cfg = 0; cfg < 3; ++cfg) g = std::max(g, (size_t)sell_grid(h, cfg, h->sel[w].nchunks));
      return g;
    };
    const size_t redk =
        std::max({bk.size(), (size_t)h->wide_nblocks[0], (size_t)P.K.rows_grid, stg_red(0), sel_red(0)});
    const size_t redt =
        std::max({bt.size(), (size_t)h->wide_nblocks[1], (size_t)P.KT.rows_grid, stg_red(1), sel_red(1)});
    h->red_k = redk;
    h->red_t = redt;
    P.partA = h->dalloc<double>(redt);
    P.partB = h->dalloc<double>(2 * redk);
    P.partE0 = h->dalloc<double>(4 * (size_t)kElemBlocks);
    P.partE1 = h->dalloc<double>(10 * redk);
    P.partE2 = h->dalloc<double>(8 * redt);
    if (P.infeas) {
      P.partE3 = h->dalloc<double>(8 * redk);
      P.partE4 = h->dalloc<double>(12 * redt);
    }
    h->st = h->dalloc<DevState>(1);
    P.st = h->st;
    P.cnorm0 = std::sqrt(hred[0]);
    P.qnorm0 = std::sqrt(hred[1]);
    for (int k = 0; k < 2; ++k) {
      void* hp = nullptr;
      check(hipHostMalloc(&hp, sizeof(DevState), hipHostMallocDefault), "hipHostMalloc");
      h->host_allocs.push_back(hp);
      h->st_host[k] = static_cast<DevState*>(hp);
      check(hipEventCreateWithFlags(&h->ev[k], hipEventDisableTiming), "hipEventCreate");
    }
    check(hipStreamSynchronize(s), "setup sync");
    check(hipGetLastError(), "setup kernels");
    choose_layouts(h);
  } catch (const HipFail& f) {
    return create_failed(h, f);
  }
  h->setup_s = now_s() - t0;
  *out = h;
  return PDLP_OK;
}

extern "C" int pdlp_presolve(const pdlp_problem* p, int32_t* status, uint8_t* keep_row, uint8_t* keep_col,
                             double* lo, double* hi, double* x_fixed, double* b_reduced, double* offset) {
  if (!p) return fail(nullptr, PDLP_ERR_ARG, "NULL problem");
  std::string why;
  HostLP H;
  if (int rc = load_problem(p, nullptr, H, why)) return fail(nullptr, rc, why);
  Presolve P;
  HostLP R;
  const int st = presolve_lp(H, R, P);
  if (status) *status = st;
  const size_t m = (size_t)H.m, n = (size_t)H.n;
  if (keep_row) for (size_t i = 0; i < m && i < P.row_on.size(); ++i) keep_row[i] = P.row_on[i];
  if (keep_col) for (size_t j = 0; j < n && j < P.col_on.size(); ++j) keep_col[j] = P.col_on[j];
  if (lo) std::memcpy(lo, P.lo.data(), n * 8);
  if (hi) std::memcpy(hi, P.hi.data(), n * 8);
  if (x_fixed) std::memcpy(x_fixed, P.xfix.data(), n * 8);
  if (b_reduced && !P.b.empty()) std::memcpy(b_reduced, P.b.data(), m * 8);
  if (offset) *offset = P.offset;
  return PDLP_OK;
}

extern "C" int pdlp_set_warm_start(pdlp_handle* h, const double* x0, const double* y0, double omega0) {
  if (!h) return PDLP_ERR_ARG;
  if (h->count) return fail(h, PDLP_ERR_STATE, "pdlp_set_warm_start on a batch handle (use the _batch entry points)");
  const int32_t un = h->presolved ? h->orig.n : h->n, um = h->presolved ? h->orig.m : h->m;
  if (x0)
    for (int32_t j = 0; j < un; ++j)
      if (!std::isfinite(x0[j])) return fail(h, PDLP_ERR_DATA, "warm-start x0 is not finite");
  if (y0)
    for (int32_t i = 0; i < um; ++i)
      if (!std::isfinite(y0[i])) return fail(h, PDLP_ERR_DATA, "warm-start y0 is not finite");
  // with presolve, the kept columns' and rows' entries start the reduced LP
  std::vector<double> rx, ry;
  if (h->presolved) {
    if (x0) {
      for (int32_t j : h->pre.cols) rx.push_back(x0[j]);
      x0 = rx.data();
    }
    if (y0) {
      for (int32_t i : h->pre.rows) ry.push_back(y0[i]);
      ry.push_back(0.0);
      y0 = ry.data();
    }
  }
  if (std::isnan(omega0) || std::isinf(omega0)) return fail(h, PDLP_ERR_DATA, "warm-start omega0 is not finite");
  try {
    // x0 == NULL: zero start for x; y0 == NULL: zero start for y
    std::vector<double> zx((size_t)h->n, 0.0), zy((size_t)std::max(h->m, 1), 0.0);
    if (y0 && !h->rperm.empty()) {
      h->rows_to_dev(y0, zy.data());
      y0 = zy.data();
    }
    if (x0 && !h->cperm.empty()) {
      h->cols_to_dev(x0, zx.data());
      x0 = zx.data();
    }
    check(hipMemcpy(h->wx, x0 ? x0 : zx.data(), (size_t)h->n * 8, hipMemcpyHostToDevice), "upload x0");
    if (h->m) check(hipMemcpy(h->wy, y0 ? y0 : zy.data(), (size_t)h->m * 8, hipMemcpyHostToDevice), "upload y0");
  } catch (const HipFail& f) {
    return fail(h, PDLP_ERR_HIP, hip_msg(f));
  }
  h->has_warm = (x0 != nullptr) || (y0 != nullptr);
  h->warm_omega = omega0 > 0.0 ? omega0 : 0.0;
  return PDLP_OK;
}

// Reset the device state and run the starting-point evaluation (eager launches).
static void start_solve(pdlp_handle* h) {
  hipStream_t s = h->stream;
  DevState* s0 = h->st_host[0];
  std::memset(s0, 0, sizeof(DevState));
  s0->eta = h->eta0;
  s0->eta_hat = h->eta0;
  s0->omega = h->warm_omega > 0.0 ? h->warm_omega : h->omega0;
  s0->initial = 1;
  s0->need_eval = 1;
  s0->eps_rel = h->opt.eps_rel;
  s0->max_iter = h->opt.max_iter;
  check(hipMemcpyAsync(h->st, s0, sizeof(DevState), hipMemcpyHostToDevice, s), "upload state");
  launch_init(h->P, h->has_warm ? h->wx : nullptr, h->has_warm ? h->wy : nullptr, s);
  launch_eval(h->P, s);
  check(hipGetLastError(), "launch start");
  // the state after the starting evaluation (the first poll of the solve loop)
  check(hipMemcpyAsync(s0, h->st, sizeof(DevState), hipMemcpyDeviceToHost, s), "read state");
  check(hipStreamSynchronize(s), "start sync");
}

static void finish_solve(pdlp_handle* h, double t0) {
  hipStream_t s = h->stream;
  launch_output(h->P, s);
  DevState* f = h->st_host[0];
  check(hipMemcpyAsync(f, h->st, sizeof(DevState), hipMemcpyDeviceToHost, s), "read state");
  check(hipStreamSynchronize(s), "finish sync");
  check(hipGetLastError(), "output kernels");
  pdlp_info& I = h->info;
  I.status = f->status;
  I.returned_avg = f->ret_avg;
  I.iterations = f->k;
  I.attempts = f->attempts;
  I.restarts = f->restarts;
  I.evaluations = f->evals;
  I.rel_kkt = f->rel_kkt;
  I.rel_gap = f->rel_gap;
  I.rel_pres = f->rel_p;
  I.rel_dres = f->rel_d;
  I.primal_obj = f->pobj;
  I.dual_obj = f->dobj;
  I.omega = f->omega;
  I.eta_hat = f->eta_hat;
  I.setup_s = h->setup_s;
  I.solve_s = now_s() - t0;
  auto code = [](const DevCsr& M, const DevCsr& V) {
    if (V.layout == 3) return 3 + 16 * V.stg.cfg;
    if (V.layout == 4) return 64 + 16 * V.sel.cfg;
    return (M.layout == 1 ? 1 : (M.remap ? 2 : 0)) + (M.grid > 0 ? 4 : 0) + (V.tile == kTileWide ? 8 : 0);
  };
  I.layout_k = code(h->P.K, h->P.Ks);
  I.layout_kt = code(h->P.KT, h->P.KTs);
  I.ray_source = f->ray_src;
  I.ray_obj = f->ray_obj;
  I.ray_res = f->ray_res;
  I.m_solved = h->m;
  I.n_solved = h->n;
}

extern "C" int pdlp_set_termination(pdlp_handle* h, double eps_rel, int64_t max_iter, double time_limit_s) {
  if (!h) return PDLP_ERR_ARG;
  pdlp_options o = h->opt;
  o.eps_rel = eps_rel;
  o.max_iter = max_iter;
  o.time_limit_s = time_limit_s;
  std::string why;
  if (check_options(o, why)) return fail(h, PDLP_ERR_ARG, why);
  h->opt = o;
  return PDLP_OK;
}

// Algorithm 1 on a single-LP handle with the kernel parameters h->P: the
// captured graph (use_graph) or the same kernels launched one by one.
static int solve_single(pdlp_handle* h, bool use_graph) {
  const double t0 = now_s();
  try {
    if (use_graph && !h->gexec) build_graph(h);
    if (!use_graph) {
      h->slots_per_round = h->opt.eval_period + std::max(2, h->opt.eval_period / 8);
      h->rounds = std::max(1, 64 / h->opt.eval_period);
    }
    start_solve(h);
    hipStream_t s = h->stream;
    const int per = h->opt.poll_every;
    // accepted steps one graph can take at most: an evaluation falls due after
    // every P accepted steps and the attempt slots idle until it has run
    const int64_t per_graph = (int64_t)h->opt.eval_period * h->rounds;
    const int64_t per_tail = std::min<int64_t>(kTailSlots, h->opt.eval_period);
    // pipelined polling: launch batch b, then wait for the status copied after
    // batch b-1.  A batch holds up to poll_every graphs while the step budget
    // left after the graphs in flight (each counted at the most steps it can
    // take) is positive: the full graph while that budget reaches a full
    // graph's steps, else the short one; so a solve with a step budget ends
    // with at most the idle slots of one short graph.
    int pending = -1;  // index of the status buffer of the previous batch
    int graphs_in[2] = {0, 0};     // graphs launched in the batch of each status buffer
    int64_t steps_in[2] = {0, 0};  // and the most steps they can take
    const bool done = h->st_host[0]->done != 0;
    int64_t k_seen = h->st_host[0]->k;
    int64_t in_flight = 0;       // steps the graphs launched after the status k_seen can take at most
    int cur = 0;
    int64_t last_k = -1;
    int stalls = 0;
    while (!done) {
      int nl = 0;
      int64_t steps = 0;
      for (int i = 0; i < per; ++i) {
        const int64_t left = h->opt.max_iter - k_seen - in_flight - steps;
        if (left <= 0) break;
        ++nl;
        if (use_graph && left < per_graph) {
          check(hipGraphLaunch(h->gexec_tail, s), "hipGraphLaunch");
          steps += per_tail;
        } else if (use_graph) {
          check(hipGraphLaunch(h->gexec, s), "hipGraphLaunch");
          steps += per_graph;
        } else {
          steps += per_graph;
          for (int r = 0; r < h->rounds; ++r) {
            for (int k = 0; k < h->slots_per_round; ++k) {
              launch_primal(h->P, s);
              launch_dual(h->P, s);
              launch_decide(h->P, s);
            }
            launch_eval(h->P, s);
          }
          check(hipGetLastError(), "eager launches");
        }
      }
      graphs_in[cur] = nl;
      steps_in[cur] = steps;
      in_flight += steps;
      check(hipMemcpyAsync(h->st_host[cur], h->st, 16, hipMemcpyDeviceToHost, s), "read status");
      check(hipEventRecord(h->ev[cur], s), "hipEventRecord");
      if (pending >= 0) {
        check(hipEventSynchronize(h->ev[pending]), "hipEventSynchronize");
        if (h->st_host[pending]->done) break;
        k_seen = h->st_host[pending]->k;
        in_flight -= steps_in[pending];
        // a healthy run accepts a step within a few attempts; a batch of graphs
        // without any accepted step means the state is broken
        if (graphs_in[pending] > 0) {
          if (k_seen == last_k) {
            if (++stalls >= 64) {
              launch_set_limit(h->st, PDLP_NUMERICAL_ERROR, s);
              break;
            }
          } else {
            stalls = 0;
            last_k = k_seen;
          }
        }
      }
      if (now_s() - t0 > h->opt.time_limit_s) {
        launch_set_limit(h->st, PDLP_TIME_LIMIT, s);
        break;
      }
      pending = cur;
      cur ^= 1;
    }
    check(hipStreamSynchronize(s), "sync");
    finish_solve(h, t0);
  } catch (const HipFail& f) {
    return fail(h, PDLP_ERR_HIP, hip_msg(f));
  }
  h->solved = true;
  return PDLP_OK;
}

extern "C" int pdlp_solve(pdlp_handle* h) {
  if (!h) return PDLP_ERR_ARG;
  if (h->count) return fail(h, PDLP_ERR_STATE, "pdlp_solve on a batch handle (use the _batch entry points)");
  return solve_single(h, h->opt.graph != 0);
}

// ---------------------------------------------------------------------------- allocation-free solve
//
// pdlp_solve_noalloc runs the same kernels as pdlp_solve, launched one by one
// (instantiating a graph allocates), with every reduction partial and segment
// sum of the solve in `scratch`, a static device array that each GPU the
// library runs on holds until the process ends.  Host code never uses the
// array's name as an address: the device address comes from
// hipGetSymbolAddress, looked up once per device on the first call there.

constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (which must be current).
hipError_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_addr[dev] = ptr;
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}
}  // namespace

extern "C" int pdlp_solve_noalloc(pdlp_handle* h) {
  if (!h) return PDLP_ERR_ARG;
  if (h->count) return fail(h, PDLP_ERR_STATE, "pdlp_solve_noalloc on a batch handle");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(h, PDLP_ERR_HIP, "hipGetDevice failed");
  if (dev != h->device)
    return fail(h, PDLP_ERR_STATE, "pdlp_solve_noalloc: make the handle's device (" + std::to_string(h->device) +
                                       ") current first (current: " + std::to_string(dev) + ")");
  if (dev < 0 || dev >= kMaxDevices) return fail(h, PDLP_ERR_UNSUPPORTED, "device index beyond 63");
  // the buffers the solve writes and reads within one step or evaluation:
  // reduction partials, and the segment sums of the layouts in use
  Params Q = h->P;
  struct Part {
    double** at[4];
    size_t count;
  };
  Part parts[16];
  int np = 0;
  auto add = [&](double** a, size_t count, double** b = nullptr) { parts[np++] = Part{{a, b, nullptr, nullptr}, count}; };
  add(&Q.partA, h->red_t);
  add(&Q.partB, 2 * h->red_k);
  add(&Q.partE0, 4 * (size_t)kElemBlocks);
  add(&Q.partE1, 10 * h->red_k);
  add(&Q.partE2, 8 * h->red_t);
  if (Q.infeas) {
    add(&Q.partE3, 8 * h->red_k);
    add(&Q.partE4, 12 * h->red_t);
  }
  if (Q.gap) add(&Q.partG, (size_t)kGapAcc * 2 * kElemBlocks);
  for (int w = 0; w < 2; ++w) {
    DevCsr& M = w ? Q.KT : Q.K;     // evaluation view
    DevCsr& V = w ? Q.KTs : Q.Ks;   // step view (its panel sums are the same buffer as M's)
    if ((M.layout == 1 || V.layout == 1) && M.pan.part)
      add(&M.pan.part, 2 * (size_t)std::max(M.pan.nseg, 1), V.layout == 1 ? &V.pan.part : nullptr);
    if (V.layout == 3) {
      add(&V.stg.part, std::max<size_t>((size_t)V.stg.npan * (size_t)V.stg.rlong, 1));
      if (V.pan.part) add(&V.pan.part, (size_t)std::max(V.pan.nseg, 1));   // the short rows' panel sums
    }
  }
  size_t need = 0;
  for (int i = 0; i < np; ++i) need = (need + 255) / 256 * 256 + parts[i].count * sizeof(double);
  if (need > kScratchBytes)
    return fail(h, PDLP_ERR_UNSUPPORTED,
                "pdlp_solve_noalloc: this LP's partial sums need " + std::to_string(need) +
                    " bytes of device scratch, more than its " + std::to_string(kScratchBytes) +
                    " bytes; use pdlp_solve");
  void* base = nullptr;
  const hipError_t e = scratch_address(dev, &base);
  if (e != hipSuccess) return fail(h, PDLP_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  size_t off = 0;
  for (int i = 0; i < np; ++i) {
    const Part& q = parts[i];
    off = (off + 255) / 256 * 256;
    double* ptr = reinterpret_cast<double*>(static_cast<unsigned char*>(base) + off);
    for (double** a : q.at)
      if (a) *a = ptr;
    off += q.count * sizeof(double);
  }
  // the array keeps the last call's contents: start this solve from zeros
  if (hipMemsetAsync(base, 0, need, h->stream) != hipSuccess)
    return fail(h, PDLP_ERR_HIP, "hipMemsetAsync of the scratch failed");
  const Params saved = h->P;
  h->P = Q;
  const int rc = solve_single(h, false);
  h->P = saved;
  return rc;
}

// A device vector over the rows, in the given row order.
static void download_rows(const pdlp_handle* h, double* dst, const double* dev, const char* what) {
  if (h->rperm.empty()) {
    check(hipMemcpy(dst, dev, (size_t)h->m * 8, hipMemcpyDeviceToHost), what);
    return;
  }
  std::vector<double> t((size_t)h->m);
  check(hipMemcpy(t.data(), dev, (size_t)h->m * 8, hipMemcpyDeviceToHost), what);
  h->rows_to_given(t.data(), dst);
}

// A device vector over the columns, in the given column order.
static void download_cols(const pdlp_handle* h, double* dst, const double* dev, const char* what) {
  if (h->cperm.empty()) {
    check(hipMemcpy(dst, dev, (size_t)h->n * 8, hipMemcpyDeviceToHost), what);
    return;
  }
  std::vector<double> t((size_t)h->n);
  check(hipMemcpy(t.data(), dev, (size_t)h->n * 8, hipMemcpyDeviceToHost), what);
  h->cols_to_given(t.data(), dst);
}

extern "C" int pdlp_get_solution(pdlp_handle* h, double* x, double* y, double* rc, pdlp_info* info) {
  if (!h) return PDLP_ERR_ARG;
  if (h->count) return fail(h, PDLP_ERR_STATE, "pdlp_get_solution on a batch handle (use the _batch entry points)");
  if (!h->solved) return fail(h, PDLP_ERR_STATE, "pdlp_get_solution before pdlp_solve");
  if (h->presolved) {
    // the reduced LP's solution, postsolved to the user's LP
    const HostLP& O = h->orig;
    std::vector<double> xr((size_t)h->n), yr((size_t)std::max(h->m, 1)), lr((size_t)h->n);
    std::vector<double> xo((size_t)O.n), yo((size_t)std::max(O.m, 1)), lo((size_t)O.n);
    try {
      download_cols(h, xr.data(), h->xo, "download x");
      if (h->m) check(hipMemcpy(yr.data(), h->yo, (size_t)h->m * 8, hipMemcpyDeviceToHost), "download y");
      download_cols(h, lr.data(), h->rco, "download reduced costs");
    } catch (const HipFail& f) {
      return fail(h, PDLP_ERR_HIP, hip_msg(f));
    }
    if (!h->rperm.empty()) {
      std::vector<double> yd(yr);
      h->rows_to_given(yd.data(), yr.data());
    }
    const int st = h->info.status;
    pdlp_info I = h->info;
    if (st == PDLP_PRIMAL_INFEASIBLE) {
      // y, lambda: the dual ray extended to the user's LP (unit 2-norm again);
      // x: the current point
      std::vector<double> sx((size_t)O.n), sy((size_t)std::max(O.m, 1)), sl((size_t)O.n);
      postsolve_lp(O, h->pre, xr.data(), yr.data(), lr.data(), sx.data(), yo.data(), lo.data(), true);
      postsolve_lp(O, h->pre, xr.data(), yr.data(), lr.data(), xo.data(), sy.data(), sl.data(), false);
      double nr = 0.0;
      for (int32_t i = 0; i < O.m; ++i) nr += yo[(size_t)i] * yo[(size_t)i];
      nr = std::sqrt(nr);
      const double sc = nr > 0.0 ? 1.0 / nr : 0.0;
      for (int32_t i = 0; i < O.m; ++i) yo[(size_t)i] *= sc;
      for (int32_t j = 0; j < O.n; ++j) lo[(size_t)j] *= sc;
      I.ray_obj *= sc;
      I.ray_res *= sc;
    } else if (st == PDLP_DUAL_INFEASIBLE) {
      // x: the primal ray (removed columns cannot move); y, lambda: as solved
      std::vector<double> sx((size_t)O.n), sy((size_t)std::max(O.m, 1)), sl((size_t)O.n);
      postsolve_lp(O, h->pre, xr.data(), yr.data(), lr.data(), xo.data(), sy.data(), sl.data(), true);
      postsolve_lp(O, h->pre, xr.data(), yr.data(), lr.data(), sx.data(), yo.data(), lo.data(), false);
    } else {
      postsolve_lp(O, h->pre, xr.data(), yr.data(), lr.data(), xo.data(), yo.data(), lo.data(), false);
      I.primal_obj += h->pre.offset;
      I.dual_obj += h->pre.offset;
    }
    if (x) std::memcpy(x, xo.data(), (size_t)O.n * 8);
    if (y && O.m) std::memcpy(y, yo.data(), (size_t)O.m * 8);
    if (rc) std::memcpy(rc, lo.data(), (size_t)O.n * 8);
    if (info) *info = I;
    return PDLP_OK;
  }
  try {
    if (x) download_cols(h, x, h->xo, "download x");
    if (y && h->m) download_rows(h, y, h->yo, "download y");
    if (rc) download_cols(h, rc, h->rco, "download reduced costs");
  } catch (const HipFail& f) {
    return fail(h, PDLP_ERR_HIP, hip_msg(f));
  }
  if (info) *info = h->info;
  return PDLP_OK;
}

extern "C" int pdlp_get_iterate(pdlp_handle* h, double* x_hat, double* y_hat, pdlp_iter_state* st) {
  if (!h) return PDLP_ERR_ARG;
  if (h->count) return fail(h, PDLP_ERR_STATE, "pdlp_get_iterate on a batch handle (use the _batch entry points)");
  if (!h->solved) return fail(h, PDLP_ERR_STATE, "pdlp_get_iterate before pdlp_solve");
  if (h->presolved) return fail(h, PDLP_ERR_UNSUPPORTED, "pdlp_get_iterate on a presolved handle (the iterate is the reduced LP's)");
  try {
    DevState f;
    check(hipMemcpy(&f, h->st, sizeof f, hipMemcpyDeviceToHost), "read state");
    if (x_hat) download_cols(h, x_hat, h->P.x[f.cur], "download x~");
    if (y_hat && h->m) download_rows(h, y_hat, h->P.y[f.cur], "download y~");
    if (st) {
      st->iterations = f.k;
      st->attempts = f.attempts;
      st->restarts = f.restarts;
      st->evaluations = f.evals;
      st->eta_hat = f.eta_hat;
      st->omega = f.omega;
      st->sum_eta = f.sum_eta;
      st->kkt0 = f.kkt0;
    }
  } catch (const HipFail& f) {
    return fail(h, PDLP_ERR_HIP, hip_msg(f));
  }
  return PDLP_OK;
}

extern "C" int pdlp_get_scaling(pdlp_handle* h, double* D1, double* D2, double* val_scaled) {
  if (!h) return PDLP_ERR_ARG;
  if (h->presolved) return fail(h, PDLP_ERR_UNSUPPORTED, "pdlp_get_scaling on a presolved handle (the scaling is the reduced LP's)");
  try {
    if (D1 && h->m) download_rows(h, D1, h->D1, "download D1");
    if (D2) download_cols(h, D2, h->D2, "download D2");
    if (val_scaled && h->nnz) {
      if (h->rperm.empty()) {
        check(hipMemcpy(val_scaled, h->val, (size_t)h->nnz * 8, hipMemcpyDeviceToHost), "download K~");
      } else {
        // rows back to the given order
        std::vector<double> vd((size_t)h->nnz);
        check(hipMemcpy(vd.data(), h->val, (size_t)h->nnz * 8, hipMemcpyDeviceToHost), "download K~");
        for (size_t r = 0; r < h->rperm.size(); ++r) {
          const int32_t g0 = h->rp_given[(size_t)h->rperm[r]], d0 = h->rp_dev[r], L = h->rp_dev[r + 1] - d0;
          std::memcpy(val_scaled + g0, vd.data() + d0, (size_t)L * 8);
        }
      }
    }
  } catch (const HipFail& f) {
    return fail(h, PDLP_ERR_HIP, hip_msg(f));
  }
  return PDLP_OK;
}

extern "C" int pdlp_get_trace(pdlp_handle* h, int64_t cap, int64_t* n_att, int64_t* att_k, double* att_eta,
                              double* att_etabar, int8_t* att_acc, int64_t* n_eval, int64_t* ev_k,
                              double* ev_kkt_cur, double* ev_kkt_avg, int8_t* ev_cand, int8_t* ev_reason,
                              double* ev_omega) {
  if (!h || cap < 0) return PDLP_ERR_ARG;
  if (!h->solved) return fail(h, PDLP_ERR_STATE, "pdlp_get_trace before pdlp_solve");
  if (h->opt.trace <= 0) return fail(h, PDLP_ERR_STATE, "the handle was created with trace = 0");
  try {
    DevState f;
    check(hipMemcpy(&f, h->count ? h->bst : h->st, sizeof f, hipMemcpyDeviceToHost), "read state");
    const Trace& T = h->P.tr;
    const int64_t na = std::min<int64_t>(f.n_att, cap), ne = std::min<int64_t>(f.n_eval, cap);
    if (n_att) *n_att = na;
    if (n_eval) *n_eval = ne;
    auto cp = [&](void* dst, const void* src, int64_t cnt, size_t sz) {
      if (dst && cnt > 0) check(hipMemcpy(dst, src, (size_t)cnt * sz, hipMemcpyDeviceToHost), "download trace");
    };
    cp(att_k, T.att_k, na, 8);
    cp(att_eta, T.att_eta, na, 8);
    cp(att_etabar, T.att_etabar, na, 8);
    cp(att_acc, T.att_acc, na, 1);
    cp(ev_k, T.ev_k, ne, 8);
    cp(ev_kkt_cur, T.ev_kkt_cur, ne, 8);
    cp(ev_kkt_avg, T.ev_kkt_avg, ne, 8);
    cp(ev_cand, T.ev_cand, ne, 1);
    cp(ev_reason, T.ev_reason, ne, 1);
    cp(ev_omega, T.ev_omega, ne, 8);
  } catch (const HipFail& f) {
    return fail(h, PDLP_ERR_HIP, hip_msg(f));
  }
  return PDLP_OK;
}

extern "C" int pdlp_profile_attempts(pdlp_handle* h, int32_t attempts, double* ms_primal, double* ms_dual) {
  if (!h || attempts < 1) return PDLP_ERR_ARG;
  if (h->count) return fail(h, PDLP_ERR_STATE, "pdlp_profile_attempts on a batch handle (use the _batch entry points)");
  if (!h->solved) return fail(h, PDLP_ERR_STATE, "pdlp_profile_attempts before pdlp_solve");
  hipStream_t s = h->stream;
  const int S = h->slots_per_round > 0 ? h->slots_per_round : h->opt.eval_period + 2;
  std::vector<hipEvent_t> ev((size_t)4 * S, nullptr);
  double sa = 0.0, sb = 0.0;
  int64_t timed = 0;
  try {
    for (auto& e : ev) check(hipEventCreate(&e), "hipEventCreate");
    start_solve(h);
    DevState f;
    while (timed < attempts) {
      check(hipMemcpy(&f, h->st, sizeof f, hipMemcpyDeviceToHost), "read state");
      if (f.done) break;
      const int64_t a0 = f.attempts;
      for (int k = 0; k < S; ++k) {
        set_pass_events(ev[4 * k], ev[4 * k + 1]);
        launch_primal(h->P, s);
        set_pass_events(ev[4 * k + 2], ev[4 * k + 3]);
        launch_dual(h->P, s);
        set_pass_events(nullptr, nullptr);
        launch_decide(h->P, s);
      }
      launch_eval(h->P, s);
      check(hipStreamSynchronize(s), "sync");
      check(hipGetLastError(), "profiled launches");
      check(hipMemcpy(&f, h->st, sizeof f, hipMemcpyDeviceToHost), "read state");
      const int64_t active = std::min<int64_t>(f.attempts - a0, S);
      for (int k = 0; k < active && timed < attempts; ++k) {
        float ta = 0.f, tb = 0.f;
        check(hipEventElapsedTime(&ta, ev[4 * k], ev[4 * k + 1]), "elapsed");
        check(hipEventElapsedTime(&tb, ev[4 * k + 2], ev[4 * k + 3]), "elapsed");
        sa += ta;
        sb += tb;
        ++timed;
      }
      if (active == 0) break;
    }
  } catch (const HipFail& f) {
    set_pass_events(nullptr, nullptr);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    return fail(h, PDLP_ERR_HIP, hip_msg(f));
  }
  set_pass_events(nullptr, nullptr);
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (timed == 0) return fail(h, PDLP_ERR_STATE, "the solve finished before any attempt could be timed");
  if (ms_primal) *ms_primal = sa / (double)timed;
  if (ms_dual) *ms_dual = sb / (double)timed;
  return PDLP_OK;
}

extern "C" int pdlp_step_bytes(pdlp_handle* h, double* bytes_primal, double* bytes_dual) {
  if (!h) return PDLP_ERR_ARG;
  if (h->count) return fail(h, PDLP_ERR_STATE, "pdlp_step_bytes on a batch handle (use the _batch entry points)");
  const double sv = h->opt.a_precision == PDLP_A_FP32 ? 4.0 : 8.0;
  const double nnz = (double)h->nnz, m = (double)h->m, n = (double)h->n;
  // matrix stream + row pointers + each gathered vector once + per-row vectors
  if (bytes_primal) *bytes_primal = nnz * (sv + 4.0) + 4.0 * (n + 1) + 8.0 * m + 64.0 * n;
  if (bytes_dual) *bytes_dual = nnz * (sv + 4.0) + 4.0 * (m + 1) + 8.0 * n + 57.0 * m;
  return PDLP_OK;
}

// ---------------------------------------------------------------------------- batches of LPs

namespace {

// Bucket of a mean row length (ceil log2) and of an LP's row count; LPs of one
// (length, size) class share a lanes-per-row choice.
int length_class(double avg) {
  int c = 0;
  while (c < 12 && (double)(1 << c) < avg) ++c;
  return c;
}
int size_class(int32_t rows) { return rows < 256 ? 0 : (rows < 1024 ? 1 : 2); }

}  // namespace

// One persistent launch over `count` LPs taken in the order of `order` (all
// LPs by default); resume = 1 continues LPs that an earlier launch paused.
static void launch_batch_solve(pdlp_handle* h, double eps_rel, int64_t max_iter, double time_limit_s,
                               int64_t pause_at = 0, const int32_t* order = nullptr, int32_t count = -1,
                               int32_t resume = 0) {
  hipStream_t s = h->stream;
  BatchParams bp{};
  bp.count = count >= 0 ? count : h->count;
  bp.trace_lp = h->opt.trace > 0 ? 0 : -1;
  bp.order = order ? order : h->order;
  bp.resume = resume;
  bp.row_off = h->row_off;
  bp.col_off = h->col_off;
  bp.lanes = h->lanes;
  bp.bk = h->bk;
  bp.bk_off = h->bk_off;
  bp.bt = h->bt;
  bp.bt_off = h->bt_off;
  bp.st = h->bst;
  bp.norms = h->norms;
  bp.kmax = h->kmax;
  bp.omega_warm = h->omega_warm;
  bp.warm = h->warm;
  bp.wx = h->wx;
  bp.wy = h->wy;
  bp.queue = h->queue;
  bp.t0 = h->t0;
  const double ticks = time_limit_s * h->tick_hz;
  bp.ticks = ticks >= 1.8e19 ? 0 : (uint64_t)std::max(1.0, ticks);
  bp.max_reject = 1000;
  bp.pause_at = pause_at;
  bp.lds_m = h->lds_m;
  bp.lds_n = h->lds_n;
  bp.lds_bk = h->lds_bk;
  bp.lds_bt = h->lds_bt;
  bp.eps_rel = eps_rel;
  bp.max_iter = max_iter;
  bp.eps_zero = h->opt.eps_zero;
  check(hipMemsetAsync(h->queue, 0, sizeof(uint32_t), s), "clear queue");
  launch_batch(h->P, bp, h->grid, s);
  check(hipGetLastError(), "batch launch");
}

// Wall time (ms) of a capped solve of the LPs `sub` only (a queue of their own).
static double time_batch_subset(pdlp_handle* h, int64_t iters, int reps, const std::vector<int32_t>& sub) {
  check(hipMemcpyAsync(h->order2, sub.data(), sub.size() * 4, hipMemcpyHostToDevice, h->stream), "upload sample");
  hipEvent_t a = nullptr, b = nullptr;
  double best = 1e30;
  try {
    check(hipEventCreate(&a), "hipEventCreate");
    check(hipEventCreate(&b), "hipEventCreate");
    for (int r = 0; r < reps; ++r) {
      check(hipEventRecord(a, h->stream), "event");
      launch_batch_solve(h, 0.0, iters, 60.0, 0, h->order2, (int32_t)sub.size());
      check(hipEventRecord(b, h->stream), "event");
      check(hipEventSynchronize(b), "sync");
      float ms = 0.f;
      check(hipEventElapsedTime(&ms, a, b), "elapsed");
      best = std::min(best, (double)ms);
    }
  } catch (...) {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    throw;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return best;
}

namespace {
// Lanes-per-row choices already tuned in this process, per (device, LDS
// configuration, side, class): a later batch of the same classes skips the search.
std::mutex g_lane_mu;
std::map<std::tuple<int, size_t, int, int>, uint8_t> g_lane_cache;
}  // namespace

// Schedule of the persistent launch: lanes per row for the rows of K~ and of
// K~' of every LP, chosen per (row-length, size) class by timing capped
// solves of a sample of that class's LPs (at most one per workgroup of the
// launch, spread over the class) under each choice, and remembered for the
// process; then the number of workgroups, by timing capped solves of the whole
// batch.  Fixed values in the options skip the search.
static void tune_batch(pdlp_handle* h) {
  const int32_t cnt = h->count;
  const pdlp_options& opt = h->opt;
  std::vector<int> cls(2 * (size_t)cnt);
  h->lanes_h.assign(2 * (size_t)cnt, 1);
  for (int32_t b = 0; b < cnt; ++b) {
    const int32_t mb = h->row_off_h[b + 1] - h->row_off_h[b], nb = h->col_off_h[b + 1] - h->col_off_h[b];
    const double nz = (double)h->nnz_h[b];
    const double ak = mb > 0 ? nz / mb : 0.0, at = nz / nb;
    cls[2 * b] = 16 * length_class(ak) + size_class(mb);
    cls[2 * b + 1] = 16 * length_class(at) + size_class(nb);
    h->lanes_h[2 * b] = opt.batch_lanes > 0 ? (uint8_t)opt.batch_lanes : 0;
    h->lanes_h[2 * b + 1] = opt.batch_lanes > 0 ? (uint8_t)opt.batch_lanes : 0;
  }
  hipDeviceProp_t prop;
  int dev = 0;
  check(hipGetDevice(&dev), "hipGetDevice");
  check(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
  const int cus = std::max(1, prop.multiProcessorCount);
  const int full = cus * batch_occupancy(h->lds_bytes);
  h->grid = opt.batch_grid > 0 ? opt.batch_grid : std::min(cnt, full);
  auto upload = [&]() {
    check(hipMemcpy(h->lanes, h->lanes_h.data(), h->lanes_h.size(), hipMemcpyHostToDevice), "upload lanes");
  };
  upload();
  const bool tune_lanes = opt.batch_lanes == 0;
  if (!tune_lanes && opt.batch_grid) return;
  const int64_t iters = 64;
  {
    std::vector<int32_t> one(1, 0);
    (void)time_batch_subset(h, 8, 1, one);   // first launch: code object load
  }
  if (tune_lanes) {
    for (int side = 0; side < 2; ++side) {
      std::vector<int> classes;
      for (int32_t b = 0; b < cnt; ++b) classes.push_back(cls[2 * b + side]);
      std::sort(classes.begin(), classes.end());
      classes.erase(std::unique(classes.begin(), classes.end()), classes.end());
      for (int c : classes) {
        std::vector<int32_t> members;
        for (int32_t b = 0; b < cnt; ++b)
          if (cls[2 * b + side] == c) members.push_back(b);
        const auto key = std::make_tuple(dev, h->lds_bytes, side, c);
        int cached = -1;
        {
          std::lock_guard<std::mutex> lock(g_lane_mu);
          auto it = g_lane_cache.find(key);
          if (it != g_lane_cache.end()) cached = it->second;
        }
        uint8_t cur = h->lanes_h[2 * (size_t)members[0] + side];
        if (cached >= 0) {
          cur = (uint8_t)cached;
        } else {
          // a sample spread over the class, at most one LP per workgroup
          std::vector<int32_t> sub;
          const size_t take = std::min(members.size(), (size_t)std::max(1, h->grid));
          for (size_t i = 0; i < take; ++i) sub.push_back(members[i * members.size() / take]);
          auto set_class = [&](uint8_t L) {
            for (int32_t b : members) h->lanes_h[2 * (size_t)b + side] = L;
            upload();
          };
          double best = time_batch_subset(h, iters, 2, sub);
          const uint8_t start = cur;
          for (int L : {0, 1, 2, 4, 8, 16, 32, 64}) {
            if (L == start) continue;
            set_class((uint8_t)L);
            const double t = time_batch_subset(h, iters, 2, sub);
            if (t < 0.98 * best) {
              best = t;
              cur = (uint8_t)L;
            }
          }
          std::lock_guard<std::mutex> lock(g_lane_mu);
          g_lane_cache[key] = cur;
        }
        for (int32_t b : members) h->lanes_h[2 * (size_t)b + side] = cur;
        upload();
      }
    }
  }
  if (!opt.batch_grid) {
    std::vector<int32_t> all((size_t)cnt);
    for (int32_t b = 0; b < cnt; ++b) all[(size_t)b] = b;
    const int64_t giters = 32;
    double best = time_batch_subset(h, giters, 1, all);
    int bestg = h->grid;
    for (int g = full / 2; g >= cus; g /= 2) {
      if (g >= cnt) continue;
      h->grid = g;
      const double t = time_batch_subset(h, giters, 1, all);
      if (t < 0.98 * best) {
        best = t;
        bestg = g;
      }
    }
    h->grid = bestg;
  }
}

extern "C" int pdlp_create_batch(const pdlp_problem* ps, int32_t count, const pdlp_options* o, void* hip_stream,
                                 pdlp_handle** out) {
  if (out) *out = nullptr;
  if (!ps || !out) return fail(nullptr, PDLP_ERR_ARG, "NULL problem array or output pointer");
  if (count < 1) return fail(nullptr, PDLP_ERR_ARG, "count must be >= 1");
  pdlp_options opt;
  if (o) opt = *o;
  else pdlp_default_options(&opt);
  std::string why;
  if (check_options(opt, why)) return fail(nullptr, PDLP_ERR_ARG, why);
  if (opt.presolve) return fail(nullptr, PDLP_ERR_UNSUPPORTED, "presolve is not available for batch handles");
  const double t0 = now_s();
  HostLP H;
  std::vector<int32_t> row_off, col_off;
  std::vector<int64_t> nnz_b;
  if (int rc = pdlp::pack_problems(ps, count, hip_stream, H, row_off, col_off, nnz_b, why)) return fail(nullptr, rc, why);

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(nullptr, PDLP_ERR_HIP, "no HIP device");
  pdlp_handle* h = new pdlp_handle();
  h->m = H.m;
  h->n = H.n;
  h->nnz = H.nnz;
  h->opt = opt;
  h->stream = (hipStream_t)hip_stream;
  h->count = count;
  h->row_off_h = row_off;
  h->col_off_h = col_off;
  h->nnz_h = nnz_b;
  h->warm_h.assign((size_t)count, 0);
  h->omega_warm_h.assign((size_t)count, 0.0);
  try {
    hipStream_t s = h->stream;
    const hipMemcpyKind kind = hipMemcpyHostToDevice;
    upload_normalize_transpose(h, H);
    h->row_off = h->dalloc<int32_t>((size_t)count + 1);
    h->col_off = h->dalloc<int32_t>((size_t)count + 1);
    check(hipMemcpyAsync(h->row_off, row_off.data(), row_off.size() * 4, kind, s), "upload row offsets");
    check(hipMemcpyAsync(h->col_off, col_off.data(), col_off.size() * 4, kind, s), "upload column offsets");
    // per-LP norms in the blocked order of the single-LP path: unscaled ||q||^2, ||c||^2 ...
    h->norms = h->dalloc<double>(4 * (size_t)count);
    launch_seg_sumsq(count, h->row_off, h->q, h->norms, 4, 0, s);
    launch_seg_sumsq(count, h->col_off, h->c0, h->norms, 4, 1, s);
    scale_problem(h);
    // ... and scaled ||c~||^2, ||q~||^2, max |K~_ij|
    launch_seg_sumsq(count, h->col_off, h->c, h->norms, 4, 2, s);
    launch_seg_sumsq(count, h->row_off, h->q, h->norms, 4, 3, s);
    h->kmax = h->dalloc<double>((size_t)count);
    launch_seg_absmax(count, h->row_off, h->rp, h->val, h->kmax, s);
    check(hipGetLastError(), "per-LP norms");
    Params& P = h->P;
    P.K = DevCsr{h->rp, h->ci, h->val, h->valf, nullptr, 0, h->m, 0, 0, 0, 0, 0, PanelCsr{}};
    P.KT = DevCsr{h->rpT, h->ciT, h->valT, h->valTf, nullptr, 0, h->n, 0, 0, 0, 0, 0, PanelCsr{}};
    P.Ks = P.K;
    P.KTs = P.KT;
    alloc_iterates(h);
    P.st = nullptr;
    h->bst = h->dalloc<DevState>((size_t)count);
    h->omega_warm = h->dalloc<double>((size_t)count);
    h->warm = h->dalloc<int8_t>((size_t)count);
    h->queue = h->dalloc<uint32_t>(1);
    h->t0 = h->dalloc<uint64_t>(1);
    h->lanes = h->dalloc<uint8_t>(2 * (size_t)count);
    // LDS-tiled row blocks of every LP's rows of K~ and of K~'
    {
      std::vector<int32_t> hrpT((size_t)h->n + 1);
      check(hipMemcpy(hrpT.data(), h->rpT, ((size_t)h->n + 1) * 4, hipMemcpyDeviceToHost), "read rowptr of K'");
      std::vector<RowBlock> bk, bt;
      std::vector<int32_t> bko(1, 0), bto(1, 0);
      for (int32_t k = 0; k < count; ++k) {
        const size_t nk0 = bk.size(), nt0 = bt.size();
        const int tile = batch_tile();
        for (const RowBlock& r : partition_rows(H.rp.data(), row_off[(size_t)k], row_off[(size_t)k + 1], tile))
          bk.push_back(r);
        for (const RowBlock& r : partition_rows(hrpT.data(), col_off[(size_t)k], col_off[(size_t)k + 1], tile))
          bt.push_back(r);
        bko.push_back((int32_t)bk.size());
        bto.push_back((int32_t)bt.size());
        h->max_bk = std::max(h->max_bk, (int32_t)(bk.size() - nk0));
        h->max_bt = std::max(h->max_bt, (int32_t)(bt.size() - nt0));
      }
      h->bk = h->dalloc<RowBlock>(bk.size());
      h->bt = h->dalloc<RowBlock>(bt.size());
      h->bk_off = h->dalloc<int32_t>(bko.size());
      h->bt_off = h->dalloc<int32_t>(bto.size());
      if (!bk.empty()) check(hipMemcpy(h->bk, bk.data(), bk.size() * sizeof(RowBlock), kind), "upload blocks");
      if (!bt.empty()) check(hipMemcpy(h->bt, bt.data(), bt.size() * sizeof(RowBlock), kind), "upload blocks");
      check(hipMemcpy(h->bk_off, bko.data(), bko.size() * 4, kind), "upload block offsets");
      check(hipMemcpy(h->bt_off, bto.data(), bto.size() * 4, kind), "upload block offsets");
      // the same rows in the tiling of the single-LP kernels (for the hand-off);
      // an LP without rows gets one empty block
      bk.clear();
      bt.clear();
      h->hk_off.assign(1, 0);
      h->ht_off.assign(1, 0);
      for (int32_t k = 0; k < count; ++k) {
        const int32_t i0 = row_off[(size_t)k], i1 = row_off[(size_t)k + 1];
        const int32_t j0 = col_off[(size_t)k], j1 = col_off[(size_t)k + 1];
        std::vector<RowBlock> a = partition_rows(H.rp.data(), i0, i1);
        if (a.empty()) a.push_back(RowBlock{i0, i0});
        std::vector<RowBlock> c = partition_rows(hrpT.data(), j0, j1);
        if (c.empty()) c.push_back(RowBlock{j0, j0});
        bk.insert(bk.end(), a.begin(), a.end());
        bt.insert(bt.end(), c.begin(), c.end());
        h->hk_off.push_back((int32_t)bk.size());
        h->ht_off.push_back((int32_t)bt.size());
        h->max_hk = std::max(h->max_hk, (int32_t)a.size());
        h->max_ht = std::max(h->max_ht, (int32_t)c.size());
      }
      h->hk = h->dalloc<RowBlock>(bk.size());
      h->ht = h->dalloc<RowBlock>(bt.size());
      check(hipMemcpy(h->hk, bk.data(), bk.size() * sizeof(RowBlock), kind), "upload blocks");
      check(hipMemcpy(h->ht, bt.data(), bt.size() * sizeof(RowBlock), kind), "upload blocks");
    }
    // queue order: most nonzeros first, so that the long solves start early
    std::vector<int32_t> ord((size_t)count);
    for (int32_t k = 0; k < count; ++k) ord[(size_t)k] = k;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return nnz_b[(size_t)a] > nnz_b[(size_t)b]; });
    h->order = h->dalloc<int32_t>((size_t)count);
    h->order2 = h->dalloc<int32_t>((size_t)count);
    check(hipMemcpyAsync(h->order, ord.data(), ord.size() * 4, kind, s), "upload queue order");
    int dev = 0, khz = 0;
    check(hipGetDevice(&dev), "hipGetDevice");
    check(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev), "wall clock rate");
    h->tick_hz = 1000.0 * (khz > 0 ? khz : 100000);
    // LDS of a batch workgroup: the tile staging, plus the largest LP's y and
    // dx when they fit in what one workgroup may allocate
    {
      hipDeviceProp_t prop;
      check(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
      const size_t limit = std::max<size_t>(prop.sharedMemPerBlock, prop.sharedMemPerBlockOptin);
      const size_t stat = (size_t)batch_static_lds();
      int32_t mmax = 0, nmax = 0;
      for (int32_t k = 0; k < count; ++k) {
        mmax = std::max(mmax, row_off[(size_t)k + 1] - row_off[(size_t)k]);
        nmax = std::max(nmax, col_off[(size_t)k + 1] - col_off[(size_t)k]);
      }
      BatchParams q{};
      const size_t base = batch_lds_bytes(q);
      if (base + stat > limit)
        throw HipFail{hipErrorInvalidConfiguration, "the batched kernel's LDS tile exceeds the per-workgroup limit"};
      q.lds_m = mmax;
      q.lds_n = nmax;
      q.lds_bk = h->max_bk;
      q.lds_bt = h->max_bt;
      if (batch_lds_bytes(q) + stat <= limit && batch_prepare(batch_lds_bytes(q)) == hipSuccess) {
        h->lds_m = mmax;
        h->lds_n = nmax;
        h->lds_bk = h->max_bk;
        h->lds_bt = h->max_bt;
      } else {
        check(batch_prepare(base), "batch LDS attribute");
      }
      q.lds_m = h->lds_m;
      q.lds_n = h->lds_n;
      q.lds_bk = h->lds_bk;
      q.lds_bt = h->lds_bt;
      h->lds_bytes = batch_lds_bytes(q);
    }
    check(hipStreamSynchronize(s), "setup sync");
    check(hipGetLastError(), "setup kernels");
    h->norms_h.resize(4 * (size_t)count);
    check(hipMemcpy(h->norms_h.data(), h->norms, h->norms_h.size() * 8, hipMemcpyDeviceToHost), "read norms");
    h->handoff_h.assign((size_t)count, 0);
    tune_batch(h);
  } catch (const HipFail& f) {
    return create_failed(h, f);
  }
  h->setup_s = now_s() - t0;
  *out = h;
  return PDLP_OK;
}

extern "C" int pdlp_set_warm_start_batch(pdlp_handle* h, int32_t idx, const double* x0, const double* y0,
                                         double omega0) {
  if (!h) return PDLP_ERR_ARG;
  if (!h->count) return fail(h, PDLP_ERR_STATE, "pdlp_set_warm_start_batch on a single-LP handle");
  if (idx < -1 || idx >= h->count) return fail(h, PDLP_ERR_ARG, "idx must be -1 or in [0, count)");
  const int32_t b0 = idx < 0 ? 0 : idx, b1 = idx < 0 ? h->count : idx + 1;
  const int32_t j0 = h->col_off_h[b0], j1 = h->col_off_h[b1], i0 = h->row_off_h[b0], i1 = h->row_off_h[b1];
  if (x0)
    for (int32_t j = 0; j < j1 - j0; ++j)
      if (!std::isfinite(x0[j])) return fail(h, PDLP_ERR_DATA, "warm-start x0 is not finite");
  if (y0)
    for (int32_t i = 0; i < i1 - i0; ++i)
      if (!std::isfinite(y0[i])) return fail(h, PDLP_ERR_DATA, "warm-start y0 is not finite");
  if (std::isnan(omega0) || std::isinf(omega0)) return fail(h, PDLP_ERR_DATA, "warm-start omega0 is not finite");
  try {
    std::vector<double> zx((size_t)(j1 - j0), 0.0), zy((size_t)std::max(i1 - i0, 1), 0.0);
    check(hipMemcpy(h->wx + j0, x0 ? x0 : zx.data(), (size_t)(j1 - j0) * 8, hipMemcpyHostToDevice), "upload x0");
    if (i1 > i0)
      check(hipMemcpy(h->wy + i0, y0 ? y0 : zy.data(), (size_t)(i1 - i0) * 8, hipMemcpyHostToDevice), "upload y0");
  } catch (const HipFail& f) {
    return fail(h, PDLP_ERR_HIP, hip_msg(f));
  }
  for (int32_t b = b0; b < b1; ++b) {
    h->warm_h[(size_t)b] = (x0 != nullptr) || (y0 != nullptr);
    h->omega_warm_h[(size_t)b] = omega0 > 0.0 ? omega0 : 0.0;
  }
  return PDLP_OK;
}

// ---------------------------------------------------------------------------- hand-off

// Params of the single-LP kernels for LP b of a batch: the packed arrays, this
// LP's row blocks, its row and column ranges, its state and partials.
static Params handoff_params(const pdlp_handle* h, int32_t b, const pdlp_handle::Lane& L) {
  Params sp = h->P;
  const int32_t i0 = h->row_off_h[(size_t)b], i1 = h->row_off_h[(size_t)b + 1];
  const int32_t j0 = h->col_off_h[(size_t)b], j1 = h->col_off_h[(size_t)b + 1];
  const int32_t nk = h->hk_off[(size_t)b + 1] - h->hk_off[(size_t)b];
  const int32_t nt = h->ht_off[(size_t)b + 1] - h->ht_off[(size_t)b];
  sp.m = i1 - i0;
  sp.n = j1 - j0;
  sp.row_base = i0;
  sp.col_base = j0;
  sp.K.blocks = h->hk + h->hk_off[(size_t)b];
  sp.K.nblocks = nk;
  sp.K.nred = nk;
  sp.K.nrows = sp.m;
  sp.K.layout = sp.K.remap = sp.K.grid = 0;
  sp.K.rows_grid = elem_grid(sp.m);
  sp.KT.blocks = h->ht + h->ht_off[(size_t)b];
  sp.KT.nblocks = nt;
  sp.KT.nred = nt;
  sp.KT.nrows = sp.n;
  sp.KT.layout = sp.KT.remap = sp.KT.grid = 0;
  sp.KT.rows_grid = elem_grid(sp.n);
  sp.K.tile = sp.KT.tile = 0;   // the kTile blocks above, for every pass
  sp.Ks = sp.K;
  sp.KTs = sp.KT;
  sp.partA = L.pa;
  sp.partB = L.pb;
  sp.partE0 = L.pe0;
  sp.partE1 = L.pe1;
  sp.partE2 = L.pe2;
  sp.partE3 = L.pe3;
  sp.partE4 = L.pe4;
  sp.partG = L.pg;
  sp.st = h->bst + b;
  if (!(h->opt.trace > 0 && b == 0)) sp.tr = Trace{};
  sp.qnorm0 = std::sqrt(h->norms_h[4 * (size_t)b]);
  sp.cnorm0 = std::sqrt(h->norms_h[4 * (size_t)b + 1]);
  return sp;
}

static void handoff_lanes(pdlp_handle* h, size_t want) {
  while (h->lanes_ho.size() < want) {
    h->lanes_ho.emplace_back();
    pdlp_handle::Lane& L = h->lanes_ho.back();
    check(hipStreamCreateWithFlags(&L.s, hipStreamNonBlocking), "hipStreamCreate");
    L.pa = h->dalloc<double>((size_t)h->max_ht);
    L.pb = h->dalloc<double>(2 * (size_t)h->max_hk);
    L.pe0 = h->dalloc<double>(4 * (size_t)kElemBlocks);
    L.pe1 = h->dalloc<double>(10 * (size_t)h->max_hk);
    L.pe2 = h->dalloc<double>(8 * (size_t)h->max_ht);
    L.pg = h->dalloc<double>((size_t)kGapAcc * 2 * kElemBlocks);
    L.pe3 = h->dalloc<double>(8 * (size_t)h->max_hk);
    L.pe4 = h->dalloc<double>(12 * (size_t)h->max_ht);
    for (int k = 0; k < 2; ++k) {
      void* hp = nullptr;
      check(hipHostMalloc(&hp, sizeof(DevState), hipHostMallocDefault), "hipHostMalloc");
      h->host_allocs.push_back(hp);
      L.hst[k] = static_cast<DevState*>(hp);
      check(hipEventCreateWithFlags(&L.ev[k], hipEventDisableTiming), "hipEventCreate");
    }
  }
  if (h->opt.graph && !h->cap_stream)
    check(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
}

// Finish the LPs that the persistent launch paused (status kPaused, state in
// bst) with the single-LP kernels: the same state, ops and decisions, each LP
// on one of up to handoff_streams streams, polled as in pdlp_solve.
static void run_handoff(pdlp_handle* h, const std::vector<int32_t>& paused, double t0) {
  const size_t nl = std::min<size_t>(paused.size(), (size_t)h->opt.handoff_streams);
  handoff_lanes(h, nl);
  const int P = h->opt.eval_period;
  const int slots = P + std::max(2, P / 8), rounds = std::max(1, 64 / P);
  const int per = h->opt.poll_every;
  struct Run {
    int32_t b = -1;
    Params sp{};
    int front = 0;          // status slot of the oldest poll batch in flight
    int64_t last_k = -1;
    int stalls = 0;
  };
  std::vector<Run> run(nl);
  std::vector<hipGraph_t> graphs;
  std::vector<hipGraphExec_t> execs(nl, nullptr);
  auto cleanup = [&]() {
    for (auto& L : h->lanes_ho) (void)hipStreamSynchronize(L.s);
    for (hipGraphExec_t g : execs)
      if (g) (void)hipGraphExecDestroy(g);
    for (hipGraph_t g : graphs) (void)hipGraphDestroy(g);
  };
  auto step_round = [&](size_t l, hipStream_t s) {
    for (int r = 0; r < rounds; ++r) {
      for (int k = 0; k < slots; ++k) {
        launch_primal(run[l].sp, s);
        launch_dual(run[l].sp, s);
        launch_decide(run[l].sp, s);
      }
      launch_eval(run[l].sp, s);
    }
  };
  auto enqueue = [&](size_t l, int slot) {
    pdlp_handle::Lane& L = h->lanes_ho[l];
    for (int i = 0; i < per; ++i) {
      if (execs[l]) check(hipGraphLaunch(execs[l], L.s), "hipGraphLaunch");
      else step_round(l, L.s);
    }
    check(hipGetLastError(), "hand-off launches");
    check(hipMemcpyAsync(L.hst[slot], run[l].sp.st, 16, hipMemcpyDeviceToHost, L.s), "read status");
    check(hipEventRecord(L.ev[slot], L.s), "hipEventRecord");
  };
  auto start = [&](size_t l, int32_t b) {
    pdlp_handle::Lane& L = h->lanes_ho[l];
    if (execs[l]) {
      // the previous LP's graph may still be in flight on this stream
      check(hipStreamSynchronize(L.s), "hand-off sync");
      check(hipGraphExecDestroy(execs[l]), "hipGraphExecDestroy");
      execs[l] = nullptr;
    }
    run[l] = Run{};
    run[l].b = b;
    run[l].sp = handoff_params(h, b, L);
    h->handoff_h[(size_t)b] = h->bst_h[(size_t)b].k;
    DevState* hs = L.hst[0];
    *hs = h->bst_h[(size_t)b];
    hs->status = 0;
    hs->done = 0;
    check(hipMemcpyAsync(run[l].sp.st, hs, sizeof(DevState), hipMemcpyHostToDevice, L.s), "resume state");
    check(hipStreamSynchronize(L.s), "resume sync");
    if (h->opt.graph) {
      hipGraph_t g = nullptr;
      check(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
      step_round(l, h->cap_stream);
      check(hipStreamEndCapture(h->cap_stream, &g), "hipStreamEndCapture");
      graphs.push_back(g);
      check(hipGraphInstantiate(&execs[l], g, nullptr, nullptr, 0), "hipGraphInstantiate");
    }
    enqueue(l, 0);
    enqueue(l, 1);
    run[l].front = 0;
  };
  try {
    size_t next = 0;
    for (size_t l = 0; l < nl; ++l) start(l, paused[next++]);
    size_t active = nl;
    while (active > 0) {
      bool any = false;
      for (size_t l = 0; l < nl; ++l) {
        Run& R = run[l];
        if (R.b < 0) continue;
        pdlp_handle::Lane& L = h->lanes_ho[l];
        const hipError_t q = hipEventQuery(L.ev[R.front]);
        if (q == hipErrorNotReady) continue;
        check(q, "hipEventQuery");
        any = true;
        const DevState* hs = L.hst[R.front];
        bool fin = hs->done != 0;
        if (!fin) {
          if (hs->k == R.last_k) {
            if (++R.stalls >= 64) {
              launch_set_limit(R.sp.st, PDLP_NUMERICAL_ERROR, L.s);
              fin = true;
            }
          } else {
            R.stalls = 0;
            R.last_k = hs->k;
          }
        }
        if (!fin && now_s() - t0 > h->opt.time_limit_s) {
          launch_set_limit(R.sp.st, PDLP_TIME_LIMIT, L.s);
          fin = true;
        }
        if (!fin) {
          enqueue(l, R.front);
          R.front ^= 1;
          continue;
        }
        launch_output(R.sp, L.s);
        check(hipGetLastError(), "hand-off output");
        R.b = -1;
        if (next < paused.size()) start(l, paused[next++]);
        else --active;
      }
      if (!any) std::this_thread::yield();
    }
  } catch (...) {
    cleanup();
    throw;
  }
  cleanup();
}

extern "C" int pdlp_solve_batch(pdlp_handle* h) {
  if (!h) return PDLP_ERR_ARG;
  if (!h->count) return fail(h, PDLP_ERR_STATE, "pdlp_solve_batch on a single-LP handle");
  const double t0 = now_s();
  try {
    hipStream_t s = h->stream;
    const size_t cnt = (size_t)h->count;
    check(hipMemcpyAsync(h->warm, h->warm_h.data(), cnt, hipMemcpyHostToDevice, s), "upload warm flags");
    check(hipMemcpyAsync(h->omega_warm, h->omega_warm_h.data(), cnt * 8, hipMemcpyHostToDevice, s),
          "upload warm omegas");
    int64_t pause_at = h->opt.batch_handoff;
    launch_batch_solve(h, h->opt.eps_rel, h->opt.max_iter, h->opt.time_limit_s, pause_at);
    h->bst_h.resize(cnt);
    check(hipMemcpyAsync(h->bst_h.data(), h->bst, cnt * sizeof(DevState), hipMemcpyDeviceToHost, s), "read states");
    check(hipStreamSynchronize(s), "batch sync");
    check(hipGetLastError(), "batch kernels");
    h->handoff_h.assign(cnt, 0);
    std::vector<int32_t> paused;
    for (size_t b = 0; b < cnt; ++b)
      if (h->bst_h[b].status == kPaused) paused.push_back((int32_t)b);
    // Too many long-running LPs for the streams: continue them in the
    // persistent kernel (the same arithmetic as if they had never paused) with
    // a doubled threshold, until few enough remain for the hand-off.
    const size_t few = 8 * (size_t)h->opt.handoff_streams;
    while (paused.size() > few) {
      std::stable_sort(paused.begin(), paused.end(), [&](int32_t a, int32_t c) {
        return h->nnz_h[(size_t)a] > h->nnz_h[(size_t)c];
      });
      check(hipMemcpyAsync(h->order2, paused.data(), paused.size() * 4, hipMemcpyHostToDevice, s),
            "upload queue order");
      pause_at *= 2;
      const double left = std::max(1e-6, h->opt.time_limit_s - (now_s() - t0));
      launch_batch_solve(h, h->opt.eps_rel, h->opt.max_iter, left, pause_at, h->order2, (int32_t)paused.size(), 1);
      check(hipMemcpyAsync(h->bst_h.data(), h->bst, cnt * sizeof(DevState), hipMemcpyDeviceToHost, s),
            "read states");
      check(hipStreamSynchronize(s), "batch sync");
      check(hipGetLastError(), "batch kernels");
      std::vector<int32_t> still;
      for (int32_t b : paused)
        if (h->bst_h[(size_t)b].status == kPaused) still.push_back(b);
      paused.swap(still);
    }
    if (!paused.empty()) {
      // farthest from the tolerance first (likely the longest to finish), so
      // that those do not wait for a free stream
      std::stable_sort(paused.begin(), paused.end(), [&](int32_t a, int32_t c) {
        return h->bst_h[(size_t)a].rel_kkt > h->bst_h[(size_t)c].rel_kkt;
      });
      run_handoff(h, paused, t0);
      check(hipMemcpyAsync(h->bst_h.data(), h->bst, cnt * sizeof(DevState), hipMemcpyDeviceToHost, s),
            "read states");
      check(hipStreamSynchronize(s), "hand-off sync");
    }
  } catch (const HipFail& f) {
    return fail(h, PDLP_ERR_HIP, hip_msg(f));
  }
  h->info.solve_s = now_s() - t0;
  h->solved = true;
  return PDLP_OK;
}

extern "C" int pdlp_get_solution_batch(pdlp_handle* h, int32_t idx, double* x, double* y, double* rc,
                                       pdlp_info* info) {
  if (!h) return PDLP_ERR_ARG;
  if (!h->count) return fail(h, PDLP_ERR_STATE, "pdlp_get_solution_batch on a single-LP handle");
  if (idx < -1 || idx >= h->count) return fail(h, PDLP_ERR_ARG, "idx must be -1 or in [0, count)");
  if (!h->solved) return fail(h, PDLP_ERR_STATE, "pdlp_get_solution_batch before pdlp_solve_batch");
  const int32_t b0 = idx < 0 ? 0 : idx, b1 = idx < 0 ? h->count : idx + 1;
  const int32_t j0 = h->col_off_h[b0], j1 = h->col_off_h[b1], i0 = h->row_off_h[b0], i1 = h->row_off_h[b1];
  try {
    if (x) check(hipMemcpy(x, h->xo + j0, (size_t)(j1 - j0) * 8, hipMemcpyDeviceToHost), "download x");
    if (y && i1 > i0) check(hipMemcpy(y, h->yo + i0, (size_t)(i1 - i0) * 8, hipMemcpyDeviceToHost), "download y");
    if (rc) check(hipMemcpy(rc, h->rco + j0, (size_t)(j1 - j0) * 8, hipMemcpyDeviceToHost), "download rc");
  } catch (const HipFail& f) {
    return fail(h, PDLP_ERR_HIP, hip_msg(f));
  }
  if (info) {
    for (int32_t b = b0; b < b1; ++b) {
      const DevState& f = h->bst_h[(size_t)b];
      pdlp_info& I = info[b - b0];
      I = pdlp_info{};
      I.status = f.status;
      I.returned_avg = f.ret_avg;
      I.iterations = f.k;
      I.attempts = f.attempts;
      I.restarts = f.restarts;
      I.evaluations = f.evals;
      I.rel_kkt = f.rel_kkt;
      I.rel_gap = f.rel_gap;
      I.rel_pres = f.rel_p;
      I.rel_dres = f.rel_d;
      I.primal_obj = f.pobj;
      I.dual_obj = f.dobj;
      I.omega = f.omega;
      I.eta_hat = f.eta_hat;
      I.setup_s = h->setup_s;
      I.solve_s = h->info.solve_s;
      I.layout_k = h->lanes_h[2 * (size_t)b];
      I.layout_kt = h->lanes_h[2 * (size_t)b + 1];
      I.handoff_k = h->handoff_h[(size_t)b];
      I.ray_source = f.ray_src;
      I.ray_obj = f.ray_obj;
      I.ray_res = f.ray_res;
    }
  }
  return PDLP_OK;
}

extern "C" int pdlp_batch_schedule(pdlp_handle* h, int32_t* lanes, int32_t* grid) {
  if (!h) return PDLP_ERR_ARG;
  if (!h->count) return fail(h, PDLP_ERR_STATE, "pdlp_batch_schedule on a single-LP handle");
  if (lanes)
    for (size_t k = 0; k < h->lanes_h.size(); ++k) lanes[k] = h->lanes_h[k];
  if (grid) *grid = h->grid;
  return PDLP_OK;
}

extern "C" const char* pdlp_last_error(const pdlp_handle* h) {
  return h ? h->err.c_str() : g_create_error.c_str();
}

extern "C" void pdlp_destroy(pdlp_handle* h) {
  if (!h) return;
  h->release();
  delete h;
}
