// C ABI and host runtime of the learned warm start (include/pdlp_gnn.h).
//
// pdlp_gnn_create packs the LPs block-diagonally, transposes the packed
// constraint matrix on the device and builds the node features, edge weights,
// degrees and (optionally) scaled targets with device kernels.  A training
// step or a prediction over a range of LPs launches the forward kernels (node
// embeddings, three rounds of CSR messages + bfloat16 MFMA transforms, heads),
// then the backward kernels and Adam; the host only sequences launches and
// sums the per-LP losses of the range.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "pdlp_dev.h"
#include "pdlp_gnn.h"

namespace gnnk {
void launch_rowid(int m, const int32_t* rp, int32_t* rowid, hipStream_t s);
void launch_owner(int count, const int32_t* off, int32_t* owner, hipStream_t s);
void launch_scales(int count, const int32_t* row_off, const int32_t* col_off, const int32_t* rp, const double* c,
                   const double* b, const double* a, double* scales, hipStream_t s);
void launch_var_features(int n, const int32_t* owner, const double* scales, const double* c, const double* l,
                         const double* u, const int32_t* rpT, const double* xs, float* fv, float* invdeg, float* xt,
                         hipStream_t s);
void launch_con_features(int m, const int32_t* owner, const double* scales, const double* b, const int8_t* rt,
                         const int32_t* rp, const double* ys, float* fc, float* invdeg, float* yt, hipStream_t s);
void launch_edge_weights(int64_t nnz, const int32_t* rowid, const int32_t* owner, const double* scales,
                         const double* a, float* w, hipStream_t s);
void launch_log_omega(int count, const double* om, float* ot, hipStream_t s);
void launch_weights_bf16(const float* W, unsigned short* Wb, unsigned short* Wtb, hipStream_t s);
void launch_embed(int N, int fdim, const float* F, const float* W0, const float* b0, float* H, hipStream_t s);
void launch_spmm(bool colscale, bool acc, int N, int r0, int c0, const int32_t* rp, const int32_t* ci, const float* w,
                 const float* scale, const float* in, float* out, hipStream_t s);
void launch_gemm_fwd(int N, const float* A0, const float* A1, const unsigned short* Wt, const float* bias, float* Y,
                     hipStream_t s);
void launch_head(int N, const float* H, const float* w, const float* b, float* out, hipStream_t s);
void launch_pool(int count, const int32_t* voff, const int32_t* coff, int v0, int c0, const float* Hv,
                 const float* Hc, const float* wo, const float* bo, float* pool, float* poolpart, float* oh,
                 hipStream_t s);
void launch_loss(int count, int first, const int32_t* voff, const int32_t* coff, int v0, int c0, const float* xh,
                 const float* yh, const float* oh, const float* xt, const float* yt, const float* ot, float wx,
                 float wy, float wo, float* dxh, float* dyh, float* doh, double* loss, hipStream_t s);
void launch_predict(int nv, int nc, int v0, int c0, const int32_t* vown, const int32_t* cown, const double* scales,
                    const float* xh, const float* yh, double* x0, double* y0, hipStream_t s);
void launch_omega(int count, const float* oh, double* om, hipStream_t s);
int head_bwd_grid(int N);
void launch_head_bwd(int N, int first, const int32_t* own, const int32_t* off, const float* H, const float* dh,
                     const float* doh, const float* w, const float* wo, float* dH, float* part, hipStream_t s);
void launch_pool_bwd(int count, const float* pool, const float* doh, float* g, hipStream_t s);
void launch_gemm_dx(int N, const float* dH, const float* Hout, const unsigned short* Wb, float* D0, float* D1,
                    hipStream_t s);
void dw_shape(int N, int* rows_per_wg, int* grid);
void launch_gemm_dw(int N, int rows_per_wg, int grid, const float* A0, const float* A1, const float* dH,
                    const float* Hout, float* part, hipStream_t s);
int embed_bwd_grid(int N);
void launch_embed_bwd(int N, int fdim, const float* F, const float* dH, const float* H, float* part, hipStream_t s);
void launch_sum_parts(int nparts, int width, const float* part, float* g, hipStream_t s);
void launch_adam(int n, float* th, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t s);
}  // namespace gnnk

using namespace gnnk;

namespace {

thread_local std::string g_gnn_create_error = "no error";

struct HipFail {
  hipError_t e;
  const char* what;
};
inline void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw HipFail{e, what};
}

constexpr int kH = 64;
constexpr int kRounds = 3;
// offsets of the parameter blocks in the flat vector (see pdlp_gnn.h)
constexpr int kWv0 = 0, kWc0 = 5 * kH + kH, kRound0 = kWc0 + 4 * kH + kH;
constexpr int kRoundSize = 2 * (128 * kH + kH);
constexpr int kHeads = kRound0 + kRounds * kRoundSize;
constexpr int kWx = kHeads, kWy = kWx + kH + 1, kWo = kWy + kH + 1;
static_assert(kWo + 2 * kH + 1 == PDLP_GNN_PARAMS, "parameter layout");
inline int phi_off(int r) { return kRound0 + r * kRoundSize; }
inline int psi_off(int r) { return kRound0 + r * kRoundSize + 128 * kH + kH; }

}  // namespace

struct pdlp_gnn {
  hipStream_t stream = nullptr;
  int32_t count = 0;
  int32_t m = 0, n = 0;
  int64_t nnz = 0;
  std::vector<int32_t> row_off_h, col_off_h;
  std::vector<void*> allocs;
  int32_t *row_off = nullptr, *col_off = nullptr;
  int32_t *rp = nullptr, *ci = nullptr, *rpT = nullptr, *ciT = nullptr, *vown = nullptr, *cown = nullptr;
  float *w = nullptr, *wT = nullptr, *fv = nullptr, *fc = nullptr, *invdv = nullptr, *invdc = nullptr;
  double* scales = nullptr;
  float *xt = nullptr, *yt = nullptr, *ot = nullptr;
  bool has_targets = false;
  float loss_w[3] = {1.f, 1.f, 1.f};
  float *theta = nullptr, *grad = nullptr, *am = nullptr, *av = nullptr;
  int64_t adam_t = 0;
  unsigned short* wbf = nullptr;  // per transform (2 per round): W [128][64], then W' [64][128]
  // activations and backward buffers for up to cap_v / cap_c nodes, cap_k LPs
  int64_t cap_v = -1, cap_c = -1, cap_k = -1;
  std::vector<void*> act;
  float *hv[kRounds + 1] = {}, *hc[kRounds + 1] = {}, *mv[kRounds] = {}, *mc[kRounds] = {};
  float *dhv = nullptr, *dhv2 = nullptr, *dmv = nullptr, *dhc = nullptr, *dhc2 = nullptr, *dmc = nullptr;
  float *xh = nullptr, *yh = nullptr, *dxh = nullptr, *dyh = nullptr;
  float *oh = nullptr, *doh = nullptr, *pool = nullptr;
  float* poolpart = nullptr;   // per LP and node slice: partial sums of the pooling
  double *loss = nullptr, *x0 = nullptr, *y0 = nullptr, *om0 = nullptr;
  float* part = nullptr;
  std::string err = "no error";

  template <typename T>
  T* dalloc(size_t count, std::vector<void*>& list) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) throw HipFail{e, "hipMalloc"};
    list.push_back(p);
    e = hipMemsetAsync(p, 0, bytes, stream);
    if (e != hipSuccess) throw HipFail{e, "hipMemsetAsync"};
    return static_cast<T*>(p);
  }
  template <typename T>
  T* dalloc(size_t count) {
    return dalloc<T>(count, allocs);
  }
  void free_act() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (void* p : act) (void)hipFree(p);
    act.clear();
  }
  void release() {
    free_act();
    for (void* p : allocs) (void)hipFree(p);
    allocs.clear();
  }

  unsigned short* wb(int t) { return wbf + (size_t)t * 2 * 128 * kH; }
  unsigned short* wtb(int t) { return wbf + (size_t)t * 2 * 128 * kH + 128 * kH; }

  // make room for a range of nv variable nodes, nc constraint nodes, k LPs
  void ensure(int64_t nv, int64_t nc, int64_t k) {
    if (nv <= cap_v && nc <= cap_c && k <= cap_k) return;
    free_act();
    cap_v = std::max(nv, cap_v);
    cap_c = std::max(nc, cap_c);
    cap_k = std::max(k, cap_k);
    const size_t V = (size_t)cap_v * kH, C = (size_t)cap_c * kH;
    for (int r = 0; r <= kRounds; ++r) {
      hv[r] = dalloc<float>(V, act);
      hc[r] = dalloc<float>(C, act);
    }
    for (int r = 0; r < kRounds; ++r) {
      mv[r] = dalloc<float>(V, act);
      mc[r] = dalloc<float>(C, act);
    }
    dhv = dalloc<float>(V, act);
    dhv2 = dalloc<float>(V, act);
    dmv = dalloc<float>(V, act);
    dhc = dalloc<float>(C, act);
    dhc2 = dalloc<float>(C, act);
    dmc = dalloc<float>(C, act);
    xh = dalloc<float>(cap_v, act);
    dxh = dalloc<float>(cap_v, act);
    yh = dalloc<float>(cap_c, act);
    dyh = dalloc<float>(cap_c, act);
    oh = dalloc<float>(cap_k, act);
    doh = dalloc<float>(cap_k, act);
    pool = dalloc<float>((size_t)cap_k * 2 * kH, act);
    poolpart = dalloc<float>((size_t)cap_k * 16 * 2 * kH, act);
    loss = dalloc<double>(cap_k, act);
    x0 = dalloc<double>(cap_v, act);
    y0 = dalloc<double>(cap_c, act);
    om0 = dalloc<double>(cap_k, act);
    // partials: the weight-gradient kernel has at most 513 workgroups of
    // 128 x 64 + 64 floats; the head and embedding kernels at most 1024 of <= 384
    part = dalloc<float>(std::max<size_t>(513 * (128 * kH + kH), 1024 * 6 * kH), act);
  }
};

static int gfail(pdlp_gnn* g, int code, const std::string& msg) {
  if (g) g->err = msg;
  else g_gnn_create_error = msg;
  return code;
}
static std::string hmsg(const HipFail& f) { return std::string(f.what) + ": " + hipGetErrorString(f.e); }

extern "C" int pdlp_gnn_create(const pdlp_problem* ps, int32_t count, const double* x_star, const double* y_star,
                               const double* omega_star, void* hip_stream, pdlp_gnn** out) {
  if (out) *out = nullptr;
  if (!ps || !out) return gfail(nullptr, PDLP_ERR_ARG, "NULL problem array or output pointer");
  if (count < 1) return gfail(nullptr, PDLP_ERR_ARG, "count must be >= 1");
  const bool tg = x_star || y_star || omega_star;
  if (tg && !(x_star && y_star && omega_star))
    return gfail(nullptr, PDLP_ERR_ARG, "x_star, y_star and omega_star go together");
  pdlp::HostLP H;
  std::vector<int32_t> row_off, col_off;
  std::vector<int64_t> nnz_b;
  std::string why;
  if (int rc = pdlp::pack_problems(ps, count, hip_stream, H, row_off, col_off, nnz_b, why))
    return gfail(nullptr, rc, why);
  if (tg) {
    for (int64_t j = 0; j < H.n; ++j)
      if (!std::isfinite(x_star[j])) return gfail(nullptr, PDLP_ERR_DATA, "x_star is not finite");
    for (int64_t i = 0; i < H.m; ++i)
      if (!std::isfinite(y_star[i])) return gfail(nullptr, PDLP_ERR_DATA, "y_star is not finite");
    for (int32_t k = 0; k < count; ++k)
      if (!(omega_star[k] > 0.0) || !std::isfinite(omega_star[k]))
        return gfail(nullptr, PDLP_ERR_DATA, "omega_star must be finite and > 0");
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return gfail(nullptr, PDLP_ERR_HIP, "no HIP device");
  pdlp_gnn* g = new pdlp_gnn();
  g->stream = (hipStream_t)hip_stream;
  g->count = count;
  g->m = H.m;
  g->n = H.n;
  g->nnz = H.nnz;
  g->row_off_h = row_off;
  g->col_off_h = col_off;
  g->has_targets = tg;
  try {
    hipStream_t s = g->stream;
    const hipMemcpyKind kind = hipMemcpyHostToDevice;
    const int32_t m = H.m, n = H.n;
    const int64_t nnz = H.nnz;
    g->row_off = g->dalloc<int32_t>((size_t)count + 1);
    g->col_off = g->dalloc<int32_t>((size_t)count + 1);
    check(hipMemcpyAsync(g->row_off, row_off.data(), row_off.size() * 4, kind, s), "upload offsets");
    check(hipMemcpyAsync(g->col_off, col_off.data(), col_off.size() * 4, kind, s), "upload offsets");
    // staging of the packed LP (freed at the end of create)
    std::vector<void*> tmp;
    double* a = g->dalloc<double>((size_t)nnz, tmp);
    double* c = g->dalloc<double>(n, tmp);
    double* l = g->dalloc<double>(n, tmp);
    double* u = g->dalloc<double>(n, tmp);
    double* b = g->dalloc<double>(m, tmp);
    int8_t* rt = g->dalloc<int8_t>(m, tmp);
    int32_t* rowid = g->dalloc<int32_t>((size_t)nnz, tmp);
    int32_t* rowidT = g->dalloc<int32_t>((size_t)nnz, tmp);
    int32_t* perm = g->dalloc<int32_t>((size_t)nnz, tmp);
    double* aT = g->dalloc<double>((size_t)nnz, tmp);
    double* xs = tg ? g->dalloc<double>(n, tmp) : nullptr;
    double* ys = tg ? g->dalloc<double>(m, tmp) : nullptr;
    double* os = tg ? g->dalloc<double>(count, tmp) : nullptr;
    g->rp = g->dalloc<int32_t>((size_t)m + 1);
    g->ci = g->dalloc<int32_t>((size_t)nnz);
    g->rpT = g->dalloc<int32_t>((size_t)n + 1);
    g->ciT = g->dalloc<int32_t>((size_t)nnz);
    check(hipMemcpyAsync(g->rp, H.rp.data(), ((size_t)m + 1) * 4, kind, s), "upload row_ptr");
    if (nnz) check(hipMemcpyAsync(g->ci, H.ci.data(), (size_t)nnz * 4, kind, s), "upload col_idx");
    if (nnz) check(hipMemcpyAsync(a, H.v.data(), (size_t)nnz * 8, kind, s), "upload val");
    check(hipMemcpyAsync(c, H.c.data(), (size_t)n * 8, kind, s), "upload c");
    check(hipMemcpyAsync(l, H.l.data(), (size_t)n * 8, kind, s), "upload l");
    check(hipMemcpyAsync(u, H.u.data(), (size_t)n * 8, kind, s), "upload u");
    if (m) check(hipMemcpyAsync(b, H.b.data(), (size_t)m * 8, kind, s), "upload b");
    if (m) check(hipMemcpyAsync(rt, H.rt.data(), (size_t)m, kind, s), "upload row_type");
    if (tg) {
      check(hipMemcpyAsync(xs, x_star, (size_t)n * 8, kind, s), "upload x*");
      if (m) check(hipMemcpyAsync(ys, y_star, (size_t)m * 8, kind, s), "upload y*");
      check(hipMemcpyAsync(os, omega_star, (size_t)count * 8, kind, s), "upload omega*");
    }
    launch_rowid(m, g->rp, rowid, s);
    check(pdlp::setup_transpose(m, n, nnz, g->ci, a, rowid, g->rpT, g->ciT, aT, rowidT, perm, s), "transpose");
    g->vown = g->dalloc<int32_t>(n);
    g->cown = g->dalloc<int32_t>(m);
    launch_owner(count, g->col_off, g->vown, s);
    launch_owner(count, g->row_off, g->cown, s);
    g->scales = g->dalloc<double>(3 * (size_t)count);
    launch_scales(count, g->row_off, g->col_off, g->rp, c, b, a, g->scales, s);
    g->fv = g->dalloc<float>(5 * (size_t)n);
    g->fc = g->dalloc<float>(4 * (size_t)m);
    g->invdv = g->dalloc<float>(n);
    g->invdc = g->dalloc<float>(m);
    g->xt = g->dalloc<float>(n);
    g->yt = g->dalloc<float>(m);
    g->ot = g->dalloc<float>(count);
    launch_var_features(n, g->vown, g->scales, c, l, u, g->rpT, xs, g->fv, g->invdv, g->xt, s);
    launch_con_features(m, g->cown, g->scales, b, rt, g->rp, ys, g->fc, g->invdc, g->yt, s);
    if (tg) launch_log_omega(count, os, g->ot, s);
    g->w = g->dalloc<float>((size_t)nnz);
    g->wT = g->dalloc<float>((size_t)nnz);
    // edges of K' are owned through their row of K' (a column of K): owner = vown
    launch_edge_weights(nnz, rowid, g->cown, g->scales, a, g->w, s);
    launch_edge_weights(nnz, rowidT, g->vown, g->scales, aT, g->wT, s);
    g->theta = g->dalloc<float>(PDLP_GNN_PARAMS);
    g->grad = g->dalloc<float>(PDLP_GNN_PARAMS);
    g->am = g->dalloc<float>(PDLP_GNN_PARAMS);
    g->av = g->dalloc<float>(PDLP_GNN_PARAMS);
    g->wbf = g->dalloc<unsigned short>((size_t)2 * kRounds * 2 * 128 * kH);
    check(hipGetLastError(), "graph set-up kernels");
    check(hipStreamSynchronize(s), "set-up sync");
    for (void* p : tmp) (void)hipFree(p);
  } catch (const HipFail& f) {
    std::string msg = hmsg(f);
    g->release();
    delete g;
    return gfail(nullptr, (f.e == hipErrorOutOfMemory) ? PDLP_ERR_OOM : PDLP_ERR_HIP, msg);
  }
  *out = g;
  return PDLP_OK;
}

extern "C" int pdlp_gnn_set_params(pdlp_gnn* g, const float* theta) {
  if (!g || !theta) return PDLP_ERR_ARG;
  for (int e = 0; e < PDLP_GNN_PARAMS; ++e)
    if (!std::isfinite(theta[e])) return gfail(g, PDLP_ERR_DATA, "theta is not finite");
  try {
    check(hipMemcpyAsync(g->theta, theta, PDLP_GNN_PARAMS * 4, hipMemcpyHostToDevice, g->stream), "upload theta");
    check(hipMemsetAsync(g->am, 0, PDLP_GNN_PARAMS * 4, g->stream), "clear Adam");
    check(hipMemsetAsync(g->av, 0, PDLP_GNN_PARAMS * 4, g->stream), "clear Adam");
    check(hipStreamSynchronize(g->stream), "sync");
  } catch (const HipFail& f) {
    return gfail(g, PDLP_ERR_HIP, hmsg(f));
  }
  g->adam_t = 0;
  return PDLP_OK;
}

extern "C" int pdlp_gnn_set_loss_weights(pdlp_gnn* g, double wx, double wy, double wo) {
  if (!g) return PDLP_ERR_ARG;
  for (double w : {wx, wy, wo})
    if (!(w >= 0.0) || !std::isfinite(w)) return gfail(g, PDLP_ERR_ARG, "loss weights must be finite and >= 0");
  g->loss_w[0] = (float)wx;
  g->loss_w[1] = (float)wy;
  g->loss_w[2] = (float)wo;
  return PDLP_OK;
}

extern "C" int pdlp_gnn_get_params(pdlp_gnn* g, float* theta) {
  if (!g || !theta) return PDLP_ERR_ARG;
  try {
    check(hipMemcpyAsync(theta, g->theta, PDLP_GNN_PARAMS * 4, hipMemcpyDeviceToHost, g->stream), "download theta");
    check(hipStreamSynchronize(g->stream), "sync");
  } catch (const HipFail& f) {
    return gfail(g, PDLP_ERR_HIP, hmsg(f));
  }
  return PDLP_OK;
}

namespace {

struct Range {
  int first, K, v0, nv, c0, nc;
};

int range_of(pdlp_gnn* g, int32_t first, int32_t count, Range& R) {
  if (first < 0 || count < 1 || first > g->count - count) return PDLP_ERR_ARG;
  R.first = first;
  R.K = count;
  R.v0 = g->col_off_h[first];
  R.nv = g->col_off_h[first + count] - R.v0;
  R.c0 = g->row_off_h[first];
  R.nc = g->row_off_h[first + count] - R.c0;
  return PDLP_OK;
}

// Forward pass over a range (activations kept for the backward pass).
void forward(pdlp_gnn* g, const Range& R) {
  hipStream_t s = g->stream;
  g->ensure(R.nv, R.nc, R.K);
  const float* th = g->theta;
  for (int r = 0; r < kRounds; ++r) {
    launch_weights_bf16(th + phi_off(r), g->wb(2 * r), g->wtb(2 * r), s);
    launch_weights_bf16(th + psi_off(r), g->wb(2 * r + 1), g->wtb(2 * r + 1), s);
  }
  launch_embed(R.nv, 5, g->fv + (size_t)5 * R.v0, th + kWv0, th + kWv0 + 5 * kH, g->hv[0], s);
  launch_embed(R.nc, 4, g->fc + (size_t)4 * R.c0, th + kWc0, th + kWc0 + 4 * kH, g->hc[0], s);
  for (int r = 0; r < kRounds; ++r) {
    launch_spmm(false, false, R.nc, R.c0, R.v0, g->rp, g->ci, g->w, g->invdc, g->hv[r], g->mc[r], s);
    launch_gemm_fwd(R.nc, g->hc[r], g->mc[r], g->wtb(2 * r), th + phi_off(r) + 128 * kH, g->hc[r + 1], s);
    launch_spmm(false, false, R.nv, R.v0, R.c0, g->rpT, g->ciT, g->wT, g->invdv, g->hc[r + 1], g->mv[r], s);
    launch_gemm_fwd(R.nv, g->hv[r], g->mv[r], g->wtb(2 * r + 1), th + psi_off(r) + 128 * kH, g->hv[r + 1], s);
  }
  launch_head(R.nv, g->hv[kRounds], th + kWx, th + kWx + kH, g->xh, s);
  launch_head(R.nc, g->hc[kRounds], th + kWy, th + kWy + kH, g->yh, s);
  launch_pool(R.K, g->col_off + R.first, g->row_off + R.first, R.v0, R.c0, g->hv[kRounds], g->hc[kRounds],
              th + kWo, th + kWo + 2 * kH, g->pool, g->poolpart, g->oh, s);
}

// Weight-gradient partials of one transform, summed into grad[off ..].
void dw(pdlp_gnn* g, int N, const float* A0, const float* A1, const float* dH, const float* Hout, int off) {
  int rows = 0, grid = 0;
  dw_shape(N, &rows, &grid);
  launch_gemm_dw(N, rows, grid, A0, A1, dH, Hout, g->part, g->stream);
  launch_sum_parts(grid, 128 * kH + kH, g->part, g->grad + off, g->stream);
}

// Loss (mean over the range) and the gradient in g->grad.
double backward(pdlp_gnn* g, const Range& R) {
  hipStream_t s = g->stream;
  const float* th = g->theta;
  launch_loss(R.K, R.first, g->col_off + R.first, g->row_off + R.first, R.v0, R.c0, g->xh, g->yh, g->oh, g->xt,
              g->yt, g->ot, g->loss_w[0], g->loss_w[1], g->loss_w[2], g->dxh, g->dyh, g->doh, g->loss, s);
  // heads
  launch_head_bwd(R.nv, R.first, g->vown + R.v0, g->col_off, g->hv[kRounds], g->dxh, g->doh, th + kWx, th + kWo,
                  g->dhv, g->part, s);
  launch_sum_parts(head_bwd_grid(R.nv), kH + 1, g->part, g->grad + kWx, s);
  launch_head_bwd(R.nc, R.first, g->cown + R.c0, g->row_off, g->hc[kRounds], g->dyh, g->doh, th + kWy,
                  th + kWo + kH, g->dhc, g->part, s);
  launch_sum_parts(head_bwd_grid(R.nc), kH + 1, g->part, g->grad + kWy, s);
  launch_pool_bwd(R.K, g->pool, g->doh, g->grad + kWo, s);
  // rounds, last first
  for (int r = kRounds - 1; r >= 0; --r) {
    // variable update: hv[r+1] = relu([hv[r] | mv[r]] Psi + psi), mv[r] = W' hc[r+1] / d_v
    dw(g, R.nv, g->hv[r], g->mv[r], g->dhv, g->hv[r + 1], psi_off(r));
    launch_gemm_dx(R.nv, g->dhv, g->hv[r + 1], g->wb(2 * r + 1), g->dhv2, g->dmv, s);
    launch_spmm(true, true, R.nc, R.c0, R.v0, g->rp, g->ci, g->w, g->invdv, g->dmv, g->dhc, s);
    // constraint update: hc[r+1] = relu([hc[r] | mc[r]] Phi + phi), mc[r] = W hv[r] / d_c
    dw(g, R.nc, g->hc[r], g->mc[r], g->dhc, g->hc[r + 1], phi_off(r));
    launch_gemm_dx(R.nc, g->dhc, g->hc[r + 1], g->wb(2 * r), g->dhc2, g->dmc, s);
    launch_spmm(true, true, R.nv, R.v0, R.c0, g->rpT, g->ciT, g->wT, g->invdc, g->dmc, g->dhv2, s);
    std::swap(g->dhv, g->dhv2);
    std::swap(g->dhc, g->dhc2);
  }
  launch_embed_bwd(R.nv, 5, g->fv + (size_t)5 * R.v0, g->dhv, g->hv[0], g->part, s);
  launch_sum_parts(embed_bwd_grid(R.nv), 6 * kH, g->part, g->grad + kWv0, s);
  launch_embed_bwd(R.nc, 4, g->fc + (size_t)4 * R.c0, g->dhc, g->hc[0], g->part, s);
  launch_sum_parts(embed_bwd_grid(R.nc), 5 * kH, g->part, g->grad + kWc0, s);
  check(hipGetLastError(), "network kernels");
  std::vector<double> lk((size_t)R.K);
  check(hipMemcpyAsync(lk.data(), g->loss, (size_t)R.K * 8, hipMemcpyDeviceToHost, s), "download losses");
  check(hipStreamSynchronize(s), "sync");
  double L = 0.0;
  for (double v : lk) L += v;
  return L / R.K;
}

}  // namespace

extern "C" int pdlp_gnn_loss_grad(pdlp_gnn* g, int32_t first, int32_t count, double* loss, float* grad) {
  if (!g) return PDLP_ERR_ARG;
  Range R;
  if (range_of(g, first, count, R)) return gfail(g, PDLP_ERR_ARG, "LP range out of bounds");
  if (!g->has_targets) return gfail(g, PDLP_ERR_STATE, "the graph set has no targets");
  try {
    forward(g, R);
    const double L = backward(g, R);
    if (loss) *loss = L;
    if (grad) {
      check(hipMemcpyAsync(grad, g->grad, PDLP_GNN_PARAMS * 4, hipMemcpyDeviceToHost, g->stream), "download grad");
      check(hipStreamSynchronize(g->stream), "sync");
    }
  } catch (const HipFail& f) {
    return gfail(g, f.e == hipErrorOutOfMemory ? PDLP_ERR_OOM : PDLP_ERR_HIP, hmsg(f));
  }
  return PDLP_OK;
}

extern "C" int pdlp_gnn_train_step(pdlp_gnn* g, int32_t first, int32_t count, float lr, double* loss) {
  if (!g) return PDLP_ERR_ARG;
  Range R;
  if (range_of(g, first, count, R)) return gfail(g, PDLP_ERR_ARG, "LP range out of bounds");
  if (!g->has_targets) return gfail(g, PDLP_ERR_STATE, "the graph set has no targets");
  if (!(lr > 0.f) || !std::isfinite(lr)) return gfail(g, PDLP_ERR_ARG, "lr must be finite and > 0");
  try {
    forward(g, R);
    const double L = backward(g, R);
    if (loss) *loss = L;
    const int64_t t = ++g->adam_t;
    const double b1 = 0.9, b2 = 0.999;
    launch_adam(PDLP_GNN_PARAMS, g->theta, g->grad, g->am, g->av, lr, (float)b1, (float)b2, 1e-8f,
                (float)(1.0 - std::pow(b1, (double)t)), (float)(1.0 - std::pow(b2, (double)t)), g->stream);
    check(hipGetLastError(), "Adam");
  } catch (const HipFail& f) {
    return gfail(g, f.e == hipErrorOutOfMemory ? PDLP_ERR_OOM : PDLP_ERR_HIP, hmsg(f));
  }
  return PDLP_OK;
}

extern "C" int pdlp_gnn_predict(pdlp_gnn* g, int32_t first, int32_t count, double* x0, double* y0, double* omega0) {
  if (!g) return PDLP_ERR_ARG;
  Range R;
  if (range_of(g, first, count, R)) return gfail(g, PDLP_ERR_ARG, "LP range out of bounds");
  try {
    hipStream_t s = g->stream;
    forward(g, R);
    launch_predict(R.nv, R.nc, R.v0, R.c0, g->vown, g->cown, g->scales, g->xh, g->yh, g->x0, g->y0, s);
    launch_omega(R.K, g->oh, g->om0, s);
    check(hipGetLastError(), "network kernels");
    if (x0) check(hipMemcpyAsync(x0, g->x0, (size_t)R.nv * 8, hipMemcpyDeviceToHost, s), "download x0");
    if (y0 && R.nc) check(hipMemcpyAsync(y0, g->y0, (size_t)R.nc * 8, hipMemcpyDeviceToHost, s), "download y0");
    if (omega0) check(hipMemcpyAsync(omega0, g->om0, (size_t)R.K * 8, hipMemcpyDeviceToHost, s), "download omega0");
    check(hipStreamSynchronize(s), "sync");
  } catch (const HipFail& f) {
    return gfail(g, f.e == hipErrorOutOfMemory ? PDLP_ERR_OOM : PDLP_ERR_HIP, hmsg(f));
  }
  return PDLP_OK;
}

extern "C" const char* pdlp_gnn_last_error(const pdlp_gnn* g) {
  return g ? g->err.c_str() : g_gnn_create_error.c_str();
}

extern "C" void pdlp_gnn_destroy(pdlp_gnn* g) {
  if (!g) return;
  g->release();
  delete g;
}
