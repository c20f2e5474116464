// One-time setup kernels: >=-form normalisation, CSR transpose, Section 2.2
// preconditioning (Ruiz inf-norm passes, then Pock-Chambolle), scaled vectors,
// norms and the FP32-rounded matrix copies.
//
// The row reductions of the preconditioner run one thread per row in storage
// order, and the vector norms sum 4096-element blocks serially and then the
// block sums serially, so the scaled problem is bitwise reproducible.
#include <math.h>

#include <algorithm>
#include <utility>

#include "pdlp_dev.h"

namespace pdlp {

// LE rows a x <= b become (-a) x >= -b (eq. (primal-dual) has only >= and = rows).
__global__ void k_normalize(int m, const int32_t* __restrict__ rp, double* __restrict__ v,
                            const double* __restrict__ b, const int8_t* __restrict__ rt,
                            double* __restrict__ q, int8_t* __restrict__ ineq, int8_t* __restrict__ le,
                            int32_t* __restrict__ rowid) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    const int t = rt[i];
    const bool isle = t == 2;
    le[i] = isle;
    ineq[i] = t != 0;
    q[i] = isle ? -b[i] : b[i];
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      if (isle) v[p] = -v[p];
      rowid[p] = i;
    }
  }
}

__global__ void k_iota(int64_t nnz, int32_t* __restrict__ a) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
    a[p] = (int32_t)p;
}

__global__ void k_col_count(int64_t nnz, const int32_t* __restrict__ ci, int32_t* __restrict__ cnt) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&cnt[ci[p]], 1);
}

// K' entry q is K entry perm[q] (stable sort by column keeps rows ascending).
__global__ void k_transpose_fill(int64_t nnz, const int32_t* __restrict__ perm, const int32_t* __restrict__ rowid,
                                 const double* __restrict__ v, int32_t* __restrict__ ciT, double* __restrict__ vT) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * blockDim.x) {
    const int32_t p = perm[q];
    ciT[q] = rowid[p];
    vT[q] = v[p];
  }
}

// Row norm of one CSR matrix, one thread per row, storage order:
// mode 0: max |a|; mode 1: sum |a|^e (|a| itself when e == 1).  d = 1/sqrt(norm),
// 1 for an empty row; D *= d.
__global__ void k_row_factor(int nrows, const int32_t* __restrict__ rp, const double* __restrict__ v, int mode,
                             double e, double* __restrict__ d, double* __restrict__ D) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nrows; i += gridDim.x * blockDim.x) {
    double r = 0.0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      const double a = fabs(v[p]);
      if (mode == 0) r = a > r ? a : r;
      else r = __dadd_rn(r, e == 1.0 ? a : pow(a, e));
    }
    const double f = r > 0.0 ? 1.0 / sqrt(r) : 1.0;
    d[i] = f;
    D[i] = __dmul_rn(D[i], f);
  }
}

// a_ij *= d_row[i] * d_col[j]  (the product of the two factors is the same in
// K and K', so the two copies stay exact transposes of each other).
__global__ void k_apply_factors(int64_t nnz, const int32_t* __restrict__ rowid, const int32_t* __restrict__ ci,
                                double* __restrict__ v, const double* __restrict__ drow,
                                const double* __restrict__ dcol) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
    v[p] = __dmul_rn(v[p], __dmul_rn(drow[rowid[p]], dcol[ci[p]]));
}

// c~ = D2 c, l~ = l / D2, u~ = u / D2 ; q~ = D1 q.
__global__ void k_scale_cols(int n, const double* __restrict__ D2, const double* __restrict__ c0,
                             const double* __restrict__ l0, const double* __restrict__ u0, double* __restrict__ c,
                             double* __restrict__ l, double* __restrict__ u) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    c[j] = __dmul_rn(D2[j], c0[j]);
    l[j] = __ddiv_rn(l0[j], D2[j]);
    u[j] = __ddiv_rn(u0[j], D2[j]);
  }
}

__global__ void k_scale_rows(int m, const double* __restrict__ D1, double* __restrict__ q) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
    q[i] = __dmul_rn(D1[i], q[i]);
}

// Blocked sum of squares: one thread per 4096-element block, serial inside.
__global__ void k_sumsq_blocks(int64_t n, const double* __restrict__ a, double* __restrict__ part) {
  const int64_t nb = (n + 4095) / 4096;
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i0 = b * 4096, i1 = i0 + 4096 < n ? i0 + 4096 : n;
    double s = 0.0;
    for (int64_t i = i0; i < i1; ++i) s = __dadd_rn(s, __dmul_rn(a[i], a[i]));
    part[b] = s;
  }
}

__global__ void k_sum_serial(int64_t nb, const double* __restrict__ part, double* __restrict__ out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double s = 0.0;
    for (int64_t b = 0; b < nb; ++b) s = __dadd_rn(s, part[b]);
    *out = s;
  }
}

// max |a| over all entries (non-negative doubles order like their bit patterns).
__global__ void k_absmax(int64_t nnz, const double* __restrict__ v, unsigned long long* __restrict__ out) {
  double mx = 0.0;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x) {
    const double a = fabs(v[p]);
    mx = a > mx ? a : mx;
  }
  atomicMax(out, (unsigned long long)__double_as_longlong(mx));
}

__global__ void k_to_f32(int64_t nnz, const double* __restrict__ v, float* __restrict__ f) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
    f[p] = (float)v[p];
}

// Column-panel order of a matrix: entry q of the panel layout is entry perm[q].
__global__ void k_permute(int64_t nnz, const int32_t* __restrict__ perm, const int32_t* __restrict__ ci,
                          const double* __restrict__ v, const float* __restrict__ vf, int32_t* __restrict__ pci,
                          double* __restrict__ pv, float* __restrict__ pvf) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nnz; q += (int64_t)gridDim.x * blockDim.x) {
    const int32_t p = perm[q];
    pci[q] = ci[p];
    pv[q] = v[p];
    if (vf) pvf[q] = vf[p];
  }
}

// Values of a padded layout: entry q is entry perm[q], or a zero where perm[q] < 0.
__global__ void k_permute_values(int64_t count, const int32_t* __restrict__ perm, const double* __restrict__ v,
                                 const float* __restrict__ vf, double* __restrict__ pv, float* __restrict__ pvf) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x) {
    const int32_t p = perm[q];
    pv[q] = p >= 0 ? v[p] : 0.0;
    if (vf) pvf[q] = p >= 0 ? vf[p] : 0.0f;
  }
}

// Row renumbering: K~' entries keep their place and get the new row index;
// row vectors are gathered into the new order (new row r is old row perm[r]).
__global__ void k_rename(int64_t nnz, const int32_t* __restrict__ inv, int32_t* __restrict__ ci) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
    ci[e] = inv[ci[e]];
}

template <typename T>
__global__ void k_gather_rows(int32_t m, const int32_t* __restrict__ perm, const T* __restrict__ src,
                              T* __restrict__ dst) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x)
    dst[r] = src[perm[r]];
}

__global__ void k_fill(int64_t n, double* __restrict__ a, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

// ---------------------------------------------------------------------------- transpose: sort and scan
//
// CSR(K) -> CSR(K') is a stable sort of the nonzero positions by column (rows
// stay ascending inside each column): a least-significant-digit radix sort
// over 8-bit digits of the column index, each pass a tile histogram, an
// exclusive scan of the digit-major histogram table and a stable scatter;
// the row pointers of K' are the exclusive scan of the column counts.
// Every quantity is an integer count, so the results do not depend on the
// order of the atomic increments.

constexpr int kSortTile = 4096;               // keys per tile (one workgroup)
constexpr int kSortThreads = 256;
constexpr int kSortPer = kSortTile / kSortThreads;
constexpr int kRadix = 256;                   // 8-bit digits

// Digit counts of every tile, digit-major: hist[d * ntiles + tile].
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(int64_t n, const int32_t* __restrict__ keys, int shift,
                                                             int32_t* __restrict__ hist, int ntiles) {
  __shared__ int32_t h[kRadix];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int k = 0; k < kSortPer; ++k) {
    const int64_t i = base + k * kSortThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & (kRadix - 1)], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile: the tile is taken in chunks of kSortThreads keys
// in order; a key's place is its digit's offset for this tile, plus the keys
// of that digit in earlier chunks, in earlier wavefronts of this chunk and in
// lower lanes of its own wavefront (lanes with the same digit found by eight
// ballots, one per digit bit).
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(int64_t n, const int32_t* __restrict__ keys,
                                                                const int32_t* __restrict__ vals, int shift,
                                                                const int32_t* __restrict__ offs, int ntiles,
                                                                int32_t* __restrict__ keys_out,
                                                                int32_t* __restrict__ vals_out) {
  constexpr int kW = kSortThreads / 64;
  __shared__ int32_t run[kRadix];
  __shared__ int32_t wc[kW][kRadix];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  run[threadIdx.x] = 0;
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int k = 0; k < kSortPer; ++k) {
#pragma unroll
    for (int v = 0; v < kW; ++v) wc[v][threadIdx.x] = 0;
    __syncthreads();
    const int64_t i = base + k * kSortThreads + threadIdx.x;
    const bool valid = i < n;
    const int32_t key = valid ? keys[i] : 0;
    const int32_t val = valid ? vals[i] : 0;
    const int d = (key >> shift) & (kRadix - 1);
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t m = __ballot(valid && bit);
      same &= bit ? m : ~m;
    }
    const int rank = __popcll(same & below);
    if (valid && rank == 0) wc[w][d] = __popcll(same);
    __syncthreads();
    if (valid) {
      int32_t pos = offs[(int64_t)d * ntiles + blockIdx.x] + run[d] + rank;
      for (int v = 0; v < w; ++v) pos += wc[v][d];
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
    __syncthreads();
    int32_t add = 0;
#pragma unroll
    for (int v = 0; v < kW; ++v) add += wc[v][threadIdx.x];
    run[threadIdx.x] += add;
    __syncthreads();
  }
}

// Exclusive scan of n int32 counts, in three kernels: tile sums, a scan of
// the tile sums by one workgroup, each tile's scan from its offset.
__global__ __launch_bounds__(kSortThreads) void k_scan_tiles(int64_t n, const int32_t* __restrict__ in,
                                                             int32_t* __restrict__ sums) {
  __shared__ int32_t red[kSortThreads];
  const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)threadIdx.x * kSortPer;
  int32_t t = 0;
  for (int k = 0; k < kSortPer; ++k)
    if (base + k < n) t += in[base + k];
  red[threadIdx.x] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t s = 0;
    for (int j = 0; j < kSortThreads; ++j) s += red[j];
    sums[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(1024) void k_scan_top(int nt, int32_t* __restrict__ sums) {
  __shared__ int32_t part[1024];
  const int per = (nt + 1023) / 1024;
  const int b0 = threadIdx.x * per, b1 = min(nt, b0 + per);
  int32_t t = 0;
  for (int b = b0; b < b1; ++b) t += sums[b];
  part[threadIdx.x] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t s = 0;
    for (int j = 0; j < 1024; ++j) {
      const int32_t x = part[j];
      part[j] = s;
      s += x;
    }
  }
  __syncthreads();
  int32_t s = part[threadIdx.x];
  for (int b = b0; b < b1; ++b) {
    const int32_t x = sums[b];
    sums[b] = s;
    s += x;
  }
}

__global__ __launch_bounds__(kSortThreads) void k_scan_apply(int64_t n, const int32_t* __restrict__ in,
                                                             const int32_t* __restrict__ sums,
                                                             int32_t* __restrict__ out) {
  __shared__ int32_t pre[kSortThreads];
  const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)threadIdx.x * kSortPer;
  int32_t t = 0;
  for (int k = 0; k < kSortPer; ++k)
    if (base + k < n) t += in[base + k];
  pre[threadIdx.x] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t s = sums[blockIdx.x];
    for (int j = 0; j < kSortThreads; ++j) {
      const int32_t x = pre[j];
      pre[j] = s;
      s += x;
    }
  }
  __syncthreads();
  int32_t s = pre[threadIdx.x];
  for (int k = 0; k < kSortPer; ++k) {
    if (base + k < n) {
      const int32_t x = in[base + k];
      out[base + k] = s;
      s += x;
    }
  }
}

// ---------------------------------------------------------------------------- host side

static inline dim3 grid_for(int64_t n, int per = 256) {
  int64_t g = (n + per - 1) / per;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return dim3((unsigned)g);
}

hipError_t setup_normalize(int m, const int32_t* rp, double* v, const double* b, const int8_t* rt, double* q,
                           int8_t* ineq, int8_t* le, int32_t* rowid, hipStream_t s) {
  if (m > 0) hipLaunchKernelGGL(k_normalize, grid_for(m), dim3(256), 0, s, m, rp, v, b, rt, q, ineq, le, rowid);
  return hipGetLastError();
}

// Exclusive scan of n counts into out[0..n) (tile sums in `sums`, which holds
// ceil(n / kSortTile) entries).
static void scan_counts(int64_t n, const int32_t* in, int32_t* out, int32_t* sums, hipStream_t s) {
  if (n <= 0) return;
  const int nt = (int)((n + kSortTile - 1) / kSortTile);
  hipLaunchKernelGGL(k_scan_tiles, dim3(nt), dim3(kSortThreads), 0, s, n, in, sums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, nt, sums);
  hipLaunchKernelGGL(k_scan_apply, dim3(nt), dim3(kSortThreads), 0, s, n, in, sums, out);
}

// CSR(K) -> CSR(K'): stable sort of the nonzero positions by column (the
// radix sort above), the column counts scanned into the row pointers of K'.
hipError_t setup_transpose(int m, int n, int64_t nnz, const int32_t* ci, const double* v, const int32_t* rowid,
                           int32_t* rpT, int32_t* ciT, double* vT, int32_t* rowidT, int32_t* perm_out,
                           hipStream_t s) {
  (void)m;
  hipError_t e;
  int32_t *ka = nullptr, *kb = nullptr, *va = nullptr, *vb = nullptr, *cnt = nullptr, *hist = nullptr,
          *sums = nullptr;
  const int64_t nz = nnz > 0 ? nnz : 1;
  const int ntiles = (int)((nz + kSortTile - 1) / kSortTile);
  const int64_t nhist = (int64_t)kRadix * ntiles;
  const int64_t nsum = std::max<int64_t>((nhist + kSortTile - 1) / kSortTile, ((int64_t)n + 1 + kSortTile - 1) / kSortTile);
  if ((e = hipMalloc(&ka, nz * sizeof(int32_t))) != hipSuccess) return e;
  if ((e = hipMalloc(&kb, nz * sizeof(int32_t))) != hipSuccess) goto out;
  if ((e = hipMalloc(&va, nz * sizeof(int32_t))) != hipSuccess) goto out;
  if ((e = hipMalloc(&vb, nz * sizeof(int32_t))) != hipSuccess) goto out;
  if ((e = hipMalloc(&cnt, (size_t)(n + 1) * sizeof(int32_t))) != hipSuccess) goto out;
  if ((e = hipMalloc(&hist, (size_t)nhist * sizeof(int32_t))) != hipSuccess) goto out;
  if ((e = hipMalloc(&sums, (size_t)std::max<int64_t>(nsum, 1) * sizeof(int32_t))) != hipSuccess) goto out;
  if (nnz > 0) {
    int bits = 1;
    while (bits < 31 && (1ll << bits) < (long long)n) ++bits;
    if ((e = hipMemcpyAsync(ka, ci, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s)) != hipSuccess) goto out;
    hipLaunchKernelGGL(k_iota, grid_for(nnz), dim3(256), 0, s, nnz, va);
    for (int shift = 0; shift < bits; shift += 8) {
      hipLaunchKernelGGL(k_radix_hist, dim3(ntiles), dim3(kSortThreads), 0, s, nnz, ka, shift, hist, ntiles);
      scan_counts(nhist, hist, hist, sums, s);
      hipLaunchKernelGGL(k_radix_scatter, dim3(ntiles), dim3(kSortThreads), 0, s, nnz, ka, va, shift, hist, ntiles,
                         kb, vb);
      std::swap(ka, kb);
      std::swap(va, vb);
    }
    if ((e = hipMemcpyAsync(perm_out, va, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s)) != hipSuccess) goto out;
  }
  if ((e = hipMemsetAsync(cnt, 0, (size_t)(n + 1) * sizeof(int32_t), s)) != hipSuccess) goto out;
  if (nnz > 0) hipLaunchKernelGGL(k_col_count, grid_for(nnz), dim3(256), 0, s, nnz, ci, cnt);
  scan_counts((int64_t)n + 1, cnt, rpT, sums, s);
  if (nnz > 0) {
    hipLaunchKernelGGL(k_transpose_fill, grid_for(nnz), dim3(256), 0, s, nnz, perm_out, rowid, v, ciT, vT);
    // row ids of K' entries are the column indices of K in sorted order
    if ((e = hipMemcpyAsync(rowidT, ka, nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s)) != hipSuccess) goto out;
  }
  e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
out:
  (void)hipFree(ka);
  (void)hipFree(kb);
  (void)hipFree(va);
  (void)hipFree(vb);
  (void)hipFree(cnt);
  (void)hipFree(hist);
  (void)hipFree(sums);
  return e;
}

// Section 2.2 preconditioning on both copies.  D1, D2 must hold ones.
hipError_t setup_scale(int m, int n, int64_t nnz, const int32_t* rp, const int32_t* ci, const int32_t* rowid,
                       double* v, const int32_t* rpT, const int32_t* ciT, const int32_t* rowidT, double* vT,
                       int ruiz, double alpha, double* D1, double* D2, double* d1, double* d2, hipStream_t s) {
  const int passes = ruiz + (alpha >= 0.0 ? 1 : 0);
  for (int it = 0; it < passes; ++it) {
    const int pc = it >= ruiz;
    if (m > 0)
      hipLaunchKernelGGL(k_row_factor, grid_for(m), dim3(256), 0, s, m, rp, (const double*)v, pc, 2.0 - alpha, d1, D1);
    hipLaunchKernelGGL(k_row_factor, grid_for(n), dim3(256), 0, s, n, rpT, (const double*)vT, pc, alpha, d2, D2);
    if (nnz > 0) {
      hipLaunchKernelGGL(k_apply_factors, grid_for(nnz), dim3(256), 0, s, nnz, rowid, ci, v, (const double*)d1,
                         (const double*)d2);
      hipLaunchKernelGGL(k_apply_factors, grid_for(nnz), dim3(256), 0, s, nnz, rowidT, ciT, vT, (const double*)d2,
                         (const double*)d1);
    }
  }
  return hipGetLastError();
}

hipError_t setup_vectors(int m, int n, const double* D1, const double* D2, const double* c0, const double* l0,
                         const double* u0, double* c, double* l, double* u, double* q, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_cols, grid_for(n), dim3(256), 0, s, n, D2, c0, l0, u0, c, l, u);
  if (m > 0) hipLaunchKernelGGL(k_scale_rows, grid_for(m), dim3(256), 0, s, m, D1, q);
  return hipGetLastError();
}

// ||a||_2^2 in the blocked serial order; result written to *out (device).
hipError_t setup_sumsq(int64_t n, const double* a, double* part, double* out, hipStream_t s) {
  const int64_t nb = (n + 4095) / 4096;
  if (nb > 0) hipLaunchKernelGGL(k_sumsq_blocks, grid_for(nb, 64), dim3(64), 0, s, n, a, part);
  hipLaunchKernelGGL(k_sum_serial, dim3(1), dim3(1), 0, s, nb, (const double*)part, out);
  return hipGetLastError();
}

hipError_t setup_absmax(int64_t nnz, const double* v, unsigned long long* out, hipStream_t s) {
  hipError_t e = hipMemsetAsync(out, 0, sizeof(unsigned long long), s);
  if (e != hipSuccess) return e;
  if (nnz > 0) hipLaunchKernelGGL(k_absmax, grid_for(nnz, 1024), dim3(256), 0, s, nnz, v, out);
  return hipGetLastError();
}

hipError_t setup_to_f32(int64_t nnz, const double* v, float* f, hipStream_t s) {
  if (nnz > 0) hipLaunchKernelGGL(k_to_f32, grid_for(nnz), dim3(256), 0, s, nnz, v, f);
  return hipGetLastError();
}

hipError_t setup_permute(int64_t nnz, const int32_t* perm, const int32_t* ci, const double* v, const float* vf,
                         int32_t* pci, double* pv, float* pvf, hipStream_t s) {
  if (nnz > 0) hipLaunchKernelGGL(k_permute, grid_for(nnz), dim3(256), 0, s, nnz, perm, ci, v, vf, pci, pv, pvf);
  return hipGetLastError();
}

hipError_t setup_permute_values(int64_t count, const int32_t* perm, const double* v, const float* vf, double* pv,
                                float* pvf, hipStream_t s) {
  if (count > 0) hipLaunchKernelGGL(k_permute_values, grid_for(count), dim3(256), 0, s, count, perm, v, vf, pv, pvf);
  return hipGetLastError();
}

hipError_t setup_rename(int64_t nnz, const int32_t* inv, int32_t* ci, hipStream_t s) {
  if (nnz > 0) hipLaunchKernelGGL(k_rename, grid_for(nnz), dim3(256), 0, s, nnz, inv, ci);
  return hipGetLastError();
}

hipError_t setup_gather_rows(int32_t m, const int32_t* perm, const double* src, double* dst, hipStream_t s) {
  if (m > 0) hipLaunchKernelGGL(k_gather_rows<double>, grid_for(m), dim3(256), 0, s, m, perm, src, dst);
  return hipGetLastError();
}

hipError_t setup_gather_rows_i8(int32_t m, const int32_t* perm, const int8_t* src, int8_t* dst, hipStream_t s) {
  if (m > 0) hipLaunchKernelGGL(k_gather_rows<int8_t>, grid_for(m), dim3(256), 0, s, m, perm, src, dst);
  return hipGetLastError();
}

hipError_t setup_fill(int64_t n, double* a, double val, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill, grid_for(n), dim3(256), 0, s, n, a, val);
  return hipGetLastError();
}

}  // namespace pdlp
