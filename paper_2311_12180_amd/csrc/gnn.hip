// Kernels of the learned warm start: a bipartite message-passing network over
// the constraint graph of LPs (width 64, three rounds), its backward pass and
// Adam.  Node states are FP32 rows of 64 channels (one wavefront = one node
// row, so every gather and store is a 256-byte coalesced access).  The 128 x 64
// transforms run on the matrix cores: v_mfma_f32_16x16x32_bf16 with operands
// rounded to bfloat16 (nearest even) and FP32 accumulation.  Every reduction
// is per workgroup into a partial, then summed in a fixed order: results do not
// depend on scheduling.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace gnnk {

constexpr int kH = 64;
constexpr int kBlock = 256;

typedef __attribute__((__vector_size__(8 * sizeof(short)))) short bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ unsigned short to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// ---------------------------------------------------------------------------- set-up

// Row index of every nonzero.
__global__ void k_rowid(int m, const int32_t* __restrict__ rp, int32_t* __restrict__ rowid) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) rowid[e] = i;
}

// Owning LP of every node of a packed range.
__global__ void k_owner(int count, const int32_t* __restrict__ off, int32_t* __restrict__ owner) {
  for (int k = blockIdx.x; k < count; k += gridDim.x)
    for (int32_t i = off[k] + threadIdx.x; i < off[k + 1]; i += blockDim.x) owner[i] = k;
}

// Per-LP scales s_c = max|c|, s_b = max|b|, s_a = max|a| (1 where 0), one
// workgroup per LP.
__global__ __launch_bounds__(kBlock) void k_scales(int count, const int32_t* __restrict__ row_off,
                                                   const int32_t* __restrict__ col_off, const int32_t* __restrict__ rp,
                                                   const double* __restrict__ c, const double* __restrict__ b,
                                                   const double* __restrict__ a, double* __restrict__ scales) {
  __shared__ double red[3][kBlock / 64];
  for (int k = blockIdx.x; k < count; k += gridDim.x) {
    double mc = 0.0, mb = 0.0, ma = 0.0;
    for (int j = col_off[k] + threadIdx.x; j < col_off[k + 1]; j += kBlock) mc = fmax(mc, fabs(c[j]));
    for (int i = row_off[k] + threadIdx.x; i < row_off[k + 1]; i += kBlock) mb = fmax(mb, fabs(b[i]));
    for (int e = rp[row_off[k]] + threadIdx.x; e < rp[row_off[k + 1]]; e += kBlock) ma = fmax(ma, fabs(a[e]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      mc = fmax(mc, __shfl_down(mc, off, 64));
      mb = fmax(mb, __shfl_down(mb, off, 64));
      ma = fmax(ma, __shfl_down(ma, off, 64));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
      red[0][w] = mc;
      red[1][w] = mb;
      red[2][w] = ma;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int q = 1; q < kBlock / 64; ++q) {
        mc = fmax(mc, red[0][q]);
        mb = fmax(mb, red[1][q]);
        ma = fmax(ma, red[2][q]);
      }
      scales[3 * k] = mc > 0.0 ? mc : 1.0;
      scales[3 * k + 1] = mb > 0.0 ? mb : 1.0;
      scales[3 * k + 2] = ma > 0.0 ? ma : 1.0;
    }
    __syncthreads();
  }
}

// Variable features (5 per node), 1/degree, and the scaled target x* s_a/s_b.
__global__ void k_var_features(int n, const int32_t* __restrict__ owner, const double* __restrict__ scales,
                               const double* __restrict__ c, const double* __restrict__ l,
                               const double* __restrict__ u, const int32_t* __restrict__ rpT,
                               const double* __restrict__ xs, float* __restrict__ fv, float* __restrict__ invdeg,
                               float* __restrict__ xt) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const int k = owner[j];
    const double sc = scales[3 * k], sb = scales[3 * k + 1], sa = scales[3 * k + 2];
    const bool lf = isfinite(l[j]), uf = isfinite(u[j]);
    fv[5 * j + 0] = (float)(c[j] / sc);
    fv[5 * j + 1] = lf ? (float)(l[j] / sb) : 0.f;
    fv[5 * j + 2] = uf ? (float)(u[j] / sb) : 0.f;
    fv[5 * j + 3] = lf ? 1.f : 0.f;
    fv[5 * j + 4] = uf ? 1.f : 0.f;
    const int d = rpT[j + 1] - rpT[j];
    invdeg[j] = 1.f / (float)(d > 0 ? d : 1);
    if (xs) xt[j] = (float)(xs[j] * sa / sb);
  }
}

// Constraint features (4 per node), 1/degree, the scaled target y* s_a/s_c.
__global__ void k_con_features(int m, const int32_t* __restrict__ owner, const double* __restrict__ scales,
                               const double* __restrict__ b, const int8_t* __restrict__ rt,
                               const int32_t* __restrict__ rp, const double* __restrict__ ys,
                               float* __restrict__ fc, float* __restrict__ invdeg, float* __restrict__ yt) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    const int k = owner[i];
    const double sc = scales[3 * k], sb = scales[3 * k + 1], sa = scales[3 * k + 2];
    fc[4 * i + 0] = (float)(b[i] / sb);
    fc[4 * i + 1] = rt[i] == 0 ? 1.f : 0.f;
    fc[4 * i + 2] = rt[i] == 1 ? 1.f : 0.f;
    fc[4 * i + 3] = rt[i] == 2 ? 1.f : 0.f;
    const int d = rp[i + 1] - rp[i];
    invdeg[i] = 1.f / (float)(d > 0 ? d : 1);
    if (ys) yt[i] = (float)(ys[i] * sa / sc);
  }
}

// Edge weights a_e / s_a of the owning LP (owner indexed by the edge's row).
__global__ void k_edge_weights(int64_t nnz, const int32_t* __restrict__ rowid, const int32_t* __restrict__ owner,
                               const double* __restrict__ scales, const double* __restrict__ a,
                               float* __restrict__ w) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
    w[e] = (float)(a[e] / scales[3 * owner[rowid[e]] + 2]);
}

__global__ void k_log_omega(int count, const double* __restrict__ om, float* __restrict__ ot) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < count; k += gridDim.x * blockDim.x) ot[k] = (float)log(om[k]);
}

// bfloat16 copies of a [128][64] transform: W (same layout) and Wt ([64][128]).
__global__ void k_weights_bf16(const float* __restrict__ W, unsigned short* __restrict__ Wb,
                               unsigned short* __restrict__ Wtb) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < 128 * kH; e += gridDim.x * blockDim.x) {
    const int i = e / kH, o = e - i * kH;
    const unsigned short v = to_bf16(W[e]);
    Wb[e] = v;
    Wtb[o * 128 + i] = v;
  }
}

// ---------------------------------------------------------------------------- forward

// H[i][o] = relu(sum_k F[i][k] W0[k][o] + b0[o]) for the N nodes of a range
// (F, H start at the range), FP32.
__global__ __launch_bounds__(kBlock) void k_embed(int N, int fdim, const float* __restrict__ F,
                                                  const float* __restrict__ W0, const float* __restrict__ b0,
                                                  float* __restrict__ H) {
  const int o = threadIdx.x & 63;
  for (int i = (blockIdx.x * kBlock + threadIdx.x) >> 6; i < N; i += gridDim.x * (kBlock / 64)) {
    float z = b0[o];
    for (int k = 0; k < fdim; ++k) z += F[(size_t)i * fdim + k] * W0[k * kH + o];
    H[(size_t)i * kH + o] = z > 0.f ? z : 0.f;
  }
}

// Messages: out[r] = s_r sum_{e in row r} w_e in[col_e - c0] for rows
// [r0, r0 + N) of a CSR (global indices), s = scale[r] (ROWS) or, inside the
// sum, scale[col_e] (COLS, the adjoint of a row-scaled product).  ACC adds to
// out.  One wavefront per row, lane = channel.
template <bool COLSCALE, bool ACC>
__global__ __launch_bounds__(kBlock) void k_spmm(int N, int r0, int c0, const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ ci, const float* __restrict__ w,
                                                 const float* __restrict__ scale, const float* __restrict__ in,
                                                 float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  for (int rr = (blockIdx.x * kBlock + threadIdx.x) >> 6; rr < N; rr += gridDim.x * (kBlock / 64)) {
    const int r = r0 + rr;
    float s = 0.f;
    for (int32_t e = rp[r]; e < rp[r + 1]; ++e) {
      const int col = ci[e];
      float a = w[e];
      if (COLSCALE) a *= scale[col];
      s += a * in[(size_t)(col - c0) * kH + lane];
    }
    if (!COLSCALE) s *= scale[r];
    float* dst = out + (size_t)rr * kH + lane;
    *dst = ACC ? *dst + s : s;
  }
}

// Y[N x 64] = relu([A0 | A1] W + bias): A0, A1 [N x 64] FP32 rounded to
// bfloat16 at the load, Wt = W transposed in bfloat16 ([64][128]).  A
// workgroup of four wavefronts takes 64-row tiles; wavefront q computes rows
// 16q..16q+15 of the tile for all 64 outputs (4 column blocks x 4 k-steps).
// MFMA operand layout (16x16x32): lane l supplies A[l % 16][8 (l / 16) + 0..7]
// and B[8 (l / 16) + 0..7][l % 16]; it receives D[4 (l / 16) + 0..3][l % 16].
__global__ __launch_bounds__(kBlock) void k_gemm_fwd(int N, const float* __restrict__ A0,
                                                     const float* __restrict__ A1,
                                                     const unsigned short* __restrict__ Wt,
                                                     const float* __restrict__ bias, float* __restrict__ Y) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kg = lane >> 4;
  bf16x8 bw[4][4];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
      bw[s][nb] = *reinterpret_cast<const bf16x8*>(Wt + (16 * nb + r16) * 128 + 32 * s + 8 * kg);
  float bv[4];
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) bv[nb] = bias[16 * nb + r16];
  for (int tile = blockIdx.x; tile * 64 < N; tile += gridDim.x) {
    const int row0 = tile * 64 + wave * 16;
    const int ra = row0 + r16;
    f32x4 acc[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      bf16x8 a;
      if (ra < N) {
        const float* src = (s < 2 ? A0 : A1) + (size_t)ra * kH + (s & 1) * 32 + 8 * kg;
        const float4 v0 = *reinterpret_cast<const float4*>(src);
        const float4 v1 = *reinterpret_cast<const float4*>(src + 4);
        a[0] = (short)to_bf16(v0.x); a[1] = (short)to_bf16(v0.y); a[2] = (short)to_bf16(v0.z);
        a[3] = (short)to_bf16(v0.w); a[4] = (short)to_bf16(v1.x); a[5] = (short)to_bf16(v1.y);
        a[6] = (short)to_bf16(v1.z); a[7] = (short)to_bf16(v1.w);
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) a[q] = 0;
      }
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[s][nb], acc[nb], 0, 0, 0);
    }
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = row0 + 4 * kg + q;
        if (row < N) {
          const float z = acc[nb][q] + bv[nb];
          Y[(size_t)row * kH + 16 * nb + r16] = z > 0.f ? z : 0.f;
        }
      }
  }
}

// out[i] = H[i] . w + b (a head), one wavefront per node.
__global__ __launch_bounds__(kBlock) void k_head(int N, const float* __restrict__ H, const float* __restrict__ w,
                                                 const float* __restrict__ b, float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const float wl = w[lane];
  for (int i = (blockIdx.x * kBlock + threadIdx.x) >> 6; i < N; i += gridDim.x * (kBlock / 64)) {
    const float s = wave_sum(H[(size_t)i * kH + lane] * wl);
    if (lane == 0) out[i] = s + b[0];
  }
}

// Pooling for the omega head, pool = [mean h_v | mean h_c] per LP of the
// range and oh = pool . w_o + b_o, in two kernels so that a range of a few
// LPs still spreads over the chip: each LP's nodes are cut into kPoolSlices
// contiguous slices, one workgroup sums a slice (its wavefronts striding over
// the nodes, then added in wavefront order), and a wavefront per LP adds the
// slices in order.  voff / coff are the LPs' node offsets relative to the range.
constexpr int kPoolSlices = 16;

__global__ __launch_bounds__(kBlock) void k_pool_part(int count, const int32_t* __restrict__ voff,
                                                      const int32_t* __restrict__ coff, int v0, int c0,
                                                      const float* __restrict__ Hv, const float* __restrict__ Hc,
                                                      float* __restrict__ part) {
  __shared__ float red[2][kBlock / 64][kH];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int t = blockIdx.x; t < count * kPoolSlices; t += gridDim.x) {
    const int k = t / kPoolSlices, sl = t % kPoolSlices;
    const int jb = voff[k] - v0, je = voff[k + 1] - v0, ib = coff[k] - c0, ie = coff[k + 1] - c0;
    const int j0 = jb + (int)((int64_t)(je - jb) * sl / kPoolSlices);
    const int j1 = jb + (int)((int64_t)(je - jb) * (sl + 1) / kPoolSlices);
    const int i0 = ib + (int)((int64_t)(ie - ib) * sl / kPoolSlices);
    const int i1 = ib + (int)((int64_t)(ie - ib) * (sl + 1) / kPoolSlices);
    float sv = 0.f, sc = 0.f;
    for (int j = j0 + wave; j < j1; j += kBlock / 64) sv += Hv[(size_t)j * kH + lane];
    for (int i = i0 + wave; i < i1; i += kBlock / 64) sc += Hc[(size_t)i * kH + lane];
    red[0][wave][lane] = sv;
    red[1][wave][lane] = sc;
    __syncthreads();
    if (wave == 0) {
      float a = 0.f, c = 0.f;
      for (int q = 0; q < kBlock / 64; ++q) {
        a += red[0][q][lane];
        c += red[1][q][lane];
      }
      part[(size_t)t * 2 * kH + lane] = a;
      part[(size_t)t * 2 * kH + kH + lane] = c;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_pool_fin(int count, const int32_t* __restrict__ voff,
                                                     const int32_t* __restrict__ coff,
                                                     const float* __restrict__ part, const float* __restrict__ wo,
                                                     const float* __restrict__ bo, float* __restrict__ pool,
                                                     float* __restrict__ oh) {
  const int lane = threadIdx.x & 63;
  for (int k = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); k < count; k += gridDim.x * (kBlock / 64)) {
    const int nv = voff[k + 1] - voff[k], nc = coff[k + 1] - coff[k];
    float a = 0.f, c = 0.f;
    for (int sl = 0; sl < kPoolSlices; ++sl) {
      a += part[((size_t)k * kPoolSlices + sl) * 2 * kH + lane];
      c += part[((size_t)k * kPoolSlices + sl) * 2 * kH + kH + lane];
    }
    a = nv > 0 ? a / (float)nv : 0.f;
    c = nc > 0 ? c / (float)nc : 0.f;
    pool[(size_t)k * 128 + lane] = a;
    pool[(size_t)k * 128 + kH + lane] = c;
    const float s = wave_sum(a * wo[lane] + c * wo[kH + lane]);
    if (lane == 0) oh[k] = s + bo[0];
  }
}

// Per LP (one workgroup each): the weighted loss and the seeds of the backward
// pass, dxh = 2 w_x (xh - xt) / (n K), dyh = 2 w_y (yh - yt) / (m K),
// doh = 2 w_o (oh - ot) / K.
__global__ __launch_bounds__(kBlock) void k_loss(int count, int first, const int32_t* __restrict__ voff,
                                                 const int32_t* __restrict__ coff, int v0, int c0,
                                                 const float* __restrict__ xh, const float* __restrict__ yh,
                                                 const float* __restrict__ oh, const float* __restrict__ xt,
                                                 const float* __restrict__ yt, const float* __restrict__ ot,
                                                 float wx, float wy, float wo,
                                                 float* __restrict__ dxh, float* __restrict__ dyh,
                                                 float* __restrict__ doh, double* __restrict__ loss) {
  __shared__ double red[2][kBlock / 64];
  const float K = (float)count;
  for (int k = blockIdx.x; k < count; k += gridDim.x) {
    const int jb = voff[k] - v0, je = voff[k + 1] - v0, ib = coff[k] - c0, ie = coff[k + 1] - c0;
    const float nk = (float)(je - jb), mk = (float)(ie - ib);
    double sx = 0.0, sy = 0.0;
    for (int j = jb + threadIdx.x; j < je; j += kBlock) {
      const float d = xh[j] - xt[voff[k] + (j - jb)];
      sx += (double)d * d;
      dxh[j] = 2.f * wx * d / (nk * K);
    }
    for (int i = ib + threadIdx.x; i < ie; i += kBlock) {
      const float d = yh[i] - yt[coff[k] + (i - ib)];
      sy += (double)d * d;
      dyh[i] = 2.f * wy * d / (mk * K);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      sx += __shfl_down(sx, off, 64);
      sy += __shfl_down(sy, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      red[0][threadIdx.x >> 6] = sx;
      red[1][threadIdx.x >> 6] = sy;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double a = 0.0, c = 0.0;
      for (int q = 0; q < kBlock / 64; ++q) {
        a += red[0][q];
        c += red[1][q];
      }
      const double dw = (double)oh[k] - (double)ot[first + k];
      loss[k] = (je > jb ? (double)wx * a / (je - jb) : 0.0) + (ie > ib ? (double)wy * c / (ie - ib) : 0.0) +
                (double)wo * dw * dw;
      doh[k] = (float)(2.0 * (double)wo * dw / K);
    }
    __syncthreads();
  }
}

// Predictions in the LPs' units: x0 = xh s_b/s_a, y0 = yh s_c/s_a (owners and
// scales indexed globally, outputs relative to the range).
__global__ void k_predict(int nv, int nc, int v0, int c0, const int32_t* __restrict__ vown,
                          const int32_t* __restrict__ cown, const double* __restrict__ scales,
                          const float* __restrict__ xh, const float* __restrict__ yh, double* __restrict__ x0,
                          double* __restrict__ y0) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < nv; j += gridDim.x * blockDim.x) {
    const int k = vown[v0 + j];
    x0[j] = (double)xh[j] * scales[3 * k + 1] / scales[3 * k + 2];
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += gridDim.x * blockDim.x) {
    const int k = cown[c0 + i];
    y0[i] = (double)yh[i] * scales[3 * k] / scales[3 * k + 2];
  }
}

__global__ void k_omega(int count, const float* __restrict__ oh, double* __restrict__ om) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < count; k += gridDim.x * blockDim.x) om[k] = exp((double)oh[k]);
}

// ---------------------------------------------------------------------------- backward

// Head backward over the N nodes of a range: dH[i] = dh[i] w + doh[k(i)]
// wo / cnt(k(i)); partial (per workgroup) of sum_i dh[i] H[i] (64) and of
// sum_i dh[i] (1).  own: owner LP (global) of node i of the range; first: LP
// index of the range's first LP.
__global__ __launch_bounds__(kBlock) void k_head_bwd(int N, int first, const int32_t* __restrict__ own,
                                                     const int32_t* __restrict__ off, const float* __restrict__ H,
                                                     const float* __restrict__ dh, const float* __restrict__ doh,
                                                     const float* __restrict__ w, const float* __restrict__ wo,
                                                     float* __restrict__ dH, float* __restrict__ part) {
  __shared__ float red[kBlock / 64][kH + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float wl = w[lane], wol = wo[lane];
  float gw = 0.f, gb = 0.f;
  for (int i = (blockIdx.x * kBlock + threadIdx.x) >> 6; i < N; i += gridDim.x * (kBlock / 64)) {
    const int k = own[i] - first;
    const float cnt = (float)(off[first + k + 1] - off[first + k]);
    const float d = dh[i];
    const float h = H[(size_t)i * kH + lane];
    dH[(size_t)i * kH + lane] = d * wl + doh[k] * wol / cnt;
    gw += d * h;
    gb += d;
  }
  red[wave][lane] = gw;
  if (lane == 0) red[wave][kH] = gb;
  __syncthreads();
  if (wave == 0) {
    float a = 0.f;
    for (int q = 0; q < kBlock / 64; ++q) a += red[q][lane];
    part[(size_t)blockIdx.x * (kH + 1) + lane] = a;
    if (lane == 0) {
      float c = 0.f;
      for (int q = 0; q < kBlock / 64; ++q) c += red[q][kH];
      part[(size_t)blockIdx.x * (kH + 1) + kH] = c;
    }
  }
}

// Gradient of the omega head: g[0..127] = sum_k doh[k] pool[k], g[128] = sum_k doh[k].
__global__ void k_pool_bwd(int count, const float* __restrict__ pool, const float* __restrict__ doh,
                           float* __restrict__ g) {
  const int t = threadIdx.x;
  if (t < 129) {
    float s = 0.f;
    for (int k = 0; k < count; ++k) s += doh[k] * (t < 128 ? pool[(size_t)k * 128 + t] : 1.f);
    g[t] = s;
  }
}

// dX = dZ W' for a [128][64] transform, dZ = dH * [Hout > 0]: columns 0..63 of
// dX go to D0, 64..127 to D1 (or are added to D1 when ACC1).  W in bfloat16,
// [in][out] layout.  Same tiling and operand layout as k_gemm_fwd (K = 64:
// 2 k-steps, 8 column blocks).
__global__ __launch_bounds__(kBlock) void k_gemm_dx(int N, const float* __restrict__ dH,
                                                    const float* __restrict__ Hout,
                                                    const unsigned short* __restrict__ Wb, float* __restrict__ D0,
                                                    float* __restrict__ D1) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kg = lane >> 4;
  bf16x8 bw[2][8];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int nb = 0; nb < 8; ++nb)
      bw[s][nb] = *reinterpret_cast<const bf16x8*>(Wb + (16 * nb + r16) * kH + 32 * s + 8 * kg);
  for (int tile = blockIdx.x; tile * 64 < N; tile += gridDim.x) {
    const int row0 = tile * 64 + wave * 16;
    const int ra = row0 + r16;
    f32x4 acc[8];
#pragma unroll
    for (int nb = 0; nb < 8; ++nb) acc[nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      bf16x8 a;
      if (ra < N) {
        const size_t o = (size_t)ra * kH + 32 * s + 8 * kg;
        const float4 g0 = *reinterpret_cast<const float4*>(dH + o);
        const float4 g1 = *reinterpret_cast<const float4*>(dH + o + 4);
        const float4 h0 = *reinterpret_cast<const float4*>(Hout + o);
        const float4 h1 = *reinterpret_cast<const float4*>(Hout + o + 4);
        a[0] = (short)to_bf16(h0.x > 0.f ? g0.x : 0.f); a[1] = (short)to_bf16(h0.y > 0.f ? g0.y : 0.f);
        a[2] = (short)to_bf16(h0.z > 0.f ? g0.z : 0.f); a[3] = (short)to_bf16(h0.w > 0.f ? g0.w : 0.f);
        a[4] = (short)to_bf16(h1.x > 0.f ? g1.x : 0.f); a[5] = (short)to_bf16(h1.y > 0.f ? g1.y : 0.f);
        a[6] = (short)to_bf16(h1.z > 0.f ? g1.z : 0.f); a[7] = (short)to_bf16(h1.w > 0.f ? g1.w : 0.f);
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) a[q] = 0;
      }
#pragma unroll
      for (int nb = 0; nb < 8; ++nb) acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[s][nb], acc[nb], 0, 0, 0);
    }
#pragma unroll
    for (int nb = 0; nb < 8; ++nb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = row0 + 4 * kg + q;
        if (row < N) {
          float* dst = nb < 4 ? D0 : D1;
          dst[(size_t)row * kH + 16 * (nb & 3) + r16] = acc[nb][q];
        }
      }
  }
}

// Partial weight gradient of a [128][64] transform over rows [rb, re) of the
// range, one partial per workgroup: dW = [A0 | A1]' dZ (bfloat16 operands,
// FP32 accumulation) and db = sum dZ (FP32, unrounded), dZ = dH * [Hout > 0].
// Tiles of 32 rows are staged transposed in LDS (Xt[128][32], Zt[64][32]) so
// that each lane reads its 8 k-consecutive operands as one 16-byte access.
// Wavefront q computes the 2 x 4 output blocks of rows 32q..32q+31 of dW.
__global__ __launch_bounds__(kBlock) void k_gemm_dw(int N, int rows_per_wg, const float* __restrict__ A0,
                                                    const float* __restrict__ A1, const float* __restrict__ dH,
                                                    const float* __restrict__ Hout, float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) unsigned short Xt[128][40];
  __shared__ __attribute__((aligned(16))) unsigned short Zt[kH][40];
  __shared__ float bred[32][kH + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kg = lane >> 4;
  const int rb = blockIdx.x * rows_per_wg;
  const int re = min(N, rb + rows_per_wg);
  f32x4 acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) acc[a][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
  // staging roles: X: thread t loads row t / 8, features 16 (t % 8) .. +15;
  //                Z: thread t loads row t / 8, outputs 8 (t % 8) .. +7
  const int srow = threadIdx.x >> 3, sx = (threadIdx.x & 7) * 16, sz = (threadIdx.x & 7) * 8;
  float bsum[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) bsum[q] = 0.f;
  for (int r0 = rb; r0 < re; r0 += 32) {
    const int row = r0 + srow;
    const bool ok = row < re;
    // X: 16 features of one row (A0 for features < 64, A1 above)
    {
      const float* src = (sx < 64 ? A0 : A1) + (size_t)row * kH + (sx & 63);
#pragma unroll
      for (int q = 0; q < 16; q += 4) {
        float4 v = ok ? *reinterpret_cast<const float4*>(src + q) : float4{0.f, 0.f, 0.f, 0.f};
        Xt[sx + q + 0][srow] = to_bf16(v.x);
        Xt[sx + q + 1][srow] = to_bf16(v.y);
        Xt[sx + q + 2][srow] = to_bf16(v.z);
        Xt[sx + q + 3][srow] = to_bf16(v.w);
      }
    }
    {
      const size_t o = (size_t)row * kH + sz;
#pragma unroll
      for (int q = 0; q < 8; q += 4) {
        float4 g = ok ? *reinterpret_cast<const float4*>(dH + o + q) : float4{0.f, 0.f, 0.f, 0.f};
        float4 h = ok ? *reinterpret_cast<const float4*>(Hout + o + q) : float4{0.f, 0.f, 0.f, 0.f};
        const float z0 = h.x > 0.f ? g.x : 0.f, z1 = h.y > 0.f ? g.y : 0.f;
        const float z2 = h.z > 0.f ? g.z : 0.f, z3 = h.w > 0.f ? g.w : 0.f;
        bsum[q] += z0;
        bsum[q + 1] += z1;
        bsum[q + 2] += z2;
        bsum[q + 3] += z3;
        Zt[sz + q + 0][srow] = to_bf16(z0);
        Zt[sz + q + 1][srow] = to_bf16(z1);
        Zt[sz + q + 2][srow] = to_bf16(z2);
        Zt[sz + q + 3][srow] = to_bf16(z3);
      }
    }
    __syncthreads();
    bf16x8 bz[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) bz[nb] = *reinterpret_cast<const bf16x8*>(&Zt[16 * nb + r16][8 * kg]);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const bf16x8 ax = *reinterpret_cast<const bf16x8*>(&Xt[32 * wave + 16 * a + r16][8 * kg]);
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) acc[a][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ax, bz[nb], acc[a][nb], 0, 0, 0);
    }
    __syncthreads();
  }
  float* dst = part + (size_t)blockIdx.x * (128 * kH + kH);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb)
#pragma unroll
      for (int q = 0; q < 4; ++q) dst[(32 * wave + 16 * a + 4 * kg + q) * kH + 16 * nb + r16] = acc[a][nb][q];
  // bias: the 32 staging rows of each output column, added in row order
#pragma unroll
  for (int q = 0; q < 8; ++q) bred[srow][sz + q] = bsum[q];
  __syncthreads();
  if (threadIdx.x < kH) {
    float s = 0.f;
    for (int q = 0; q < 32; ++q) s += bred[q][threadIdx.x];
    dst[128 * kH + threadIdx.x] = s;
  }
}

// Embedding backward, one partial per workgroup: dW0[k][o] = sum_i F[i][k]
// dZ[i][o], db0[o] = sum_i dZ[i][o], dZ = dH * [H > 0].
__global__ __launch_bounds__(kBlock) void k_embed_bwd(int N, int fdim, const float* __restrict__ F,
                                                      const float* __restrict__ dH, const float* __restrict__ H,
                                                      float* __restrict__ part) {
  __shared__ float red[kBlock / 64][6][kH];
  const int o = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float acc[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int i = (blockIdx.x * kBlock + threadIdx.x) >> 6; i < N; i += gridDim.x * (kBlock / 64)) {
    const size_t e = (size_t)i * kH + o;
    const float z = H[e] > 0.f ? dH[e] : 0.f;
    for (int k = 0; k < fdim; ++k) acc[k] += F[(size_t)i * fdim + k] * z;
    acc[fdim] += z;
  }
  for (int k = 0; k <= fdim; ++k) red[wave][k][o] = acc[k];
  __syncthreads();
  if (wave == 0) {
    for (int k = 0; k <= fdim; ++k) {
      float s = 0.f;
      for (int q = 0; q < kBlock / 64; ++q) s += red[q][k][o];
      part[(size_t)blockIdx.x * ((fdim + 1) * kH) + k * kH + o] = s;
    }
  }
}

// g[e] = sum over the nparts partials of entry e: a workgroup per 64
// entries, wavefront w summing partials w, w + 4, ... (eight loads in flight),
// the four wavefront sums then added in order.
__global__ __launch_bounds__(kBlock) void k_sum_parts(int nparts, int width, const float* __restrict__ part,
                                                      float* __restrict__ g) {
  __shared__ float red[kBlock / 64][64];
  constexpr int kW = kBlock / 64;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int e0 = blockIdx.x * 64; e0 < width; e0 += gridDim.x * 64) {
    const int e = e0 + lane;
    float s = 0.f;
    if (e < width) {
      int q = w;
      for (; q + 7 * kW < nparts; q += 8 * kW) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(q + u * kW) * width + e];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
      }
      for (; q < nparts; q += kW) s += part[(size_t)q * width + e];
    }
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && e < width) {
      float t = red[0][lane];
      for (int k = 1; k < kW; ++k) t += red[k][lane];
      g[e] = t;
    }
    __syncthreads();
  }
}

// Adam step with bias correction on FP32 master weights.
__global__ void k_adam(int n, float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.f - b1) * gi;
    const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    th[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

}  // namespace gnnk

// ---------------------------------------------------------------------------- launchers

namespace gnnk {

static int grid_for(int64_t work, int per = kBlock, int cap = 8192) {
  int64_t g = (work + per - 1) / per;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

void launch_rowid(int m, const int32_t* rp, int32_t* rowid, hipStream_t s) {
  hipLaunchKernelGGL(k_rowid, dim3(grid_for(m)), dim3(kBlock), 0, s, m, rp, rowid);
}
void launch_owner(int count, const int32_t* off, int32_t* owner, hipStream_t s) {
  hipLaunchKernelGGL(k_owner, dim3(count < 8192 ? count : 8192), dim3(kBlock), 0, s, count, off, owner);
}
void launch_scales(int count, const int32_t* row_off, const int32_t* col_off, const int32_t* rp, const double* c,
                   const double* b, const double* a, double* scales, hipStream_t s) {
  hipLaunchKernelGGL(k_scales, dim3(count < 8192 ? count : 8192), dim3(kBlock), 0, s, count, row_off, col_off, rp, c,
                     b, a, scales);
}
void launch_var_features(int n, const int32_t* owner, const double* scales, const double* c, const double* l,
                         const double* u, const int32_t* rpT, const double* xs, float* fv, float* invdeg, float* xt,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_var_features, dim3(grid_for(n)), dim3(kBlock), 0, s, n, owner, scales, c, l, u, rpT, xs, fv,
                     invdeg, xt);
}
void launch_con_features(int m, const int32_t* owner, const double* scales, const double* b, const int8_t* rt,
                         const int32_t* rp, const double* ys, float* fc, float* invdeg, float* yt, hipStream_t s) {
  hipLaunchKernelGGL(k_con_features, dim3(grid_for(m)), dim3(kBlock), 0, s, m, owner, scales, b, rt, rp, ys, fc,
                     invdeg, yt);
}
void launch_edge_weights(int64_t nnz, const int32_t* rowid, const int32_t* owner, const double* scales,
                         const double* a, float* w, hipStream_t s) {
  hipLaunchKernelGGL(k_edge_weights, dim3(grid_for(nnz)), dim3(kBlock), 0, s, nnz, rowid, owner, scales, a, w);
}
void launch_log_omega(int count, const double* om, float* ot, hipStream_t s) {
  hipLaunchKernelGGL(k_log_omega, dim3(grid_for(count)), dim3(kBlock), 0, s, count, om, ot);
}
void launch_weights_bf16(const float* W, unsigned short* Wb, unsigned short* Wtb, hipStream_t s) {
  hipLaunchKernelGGL(k_weights_bf16, dim3(32), dim3(kBlock), 0, s, W, Wb, Wtb);
}
void launch_embed(int N, int fdim, const float* F, const float* W0, const float* b0, float* H, hipStream_t s) {
  hipLaunchKernelGGL(k_embed, dim3(grid_for((int64_t)N * kH)), dim3(kBlock), 0, s, N, fdim, F, W0, b0, H);
}
void launch_spmm(bool colscale, bool acc, int N, int r0, int c0, const int32_t* rp, const int32_t* ci, const float* w,
                 const float* scale, const float* in, float* out, hipStream_t s) {
  const dim3 g(grid_for((int64_t)N * kH)), b(kBlock);
  if (!colscale && !acc) hipLaunchKernelGGL((k_spmm<false, false>), g, b, 0, s, N, r0, c0, rp, ci, w, scale, in, out);
  else if (!colscale) hipLaunchKernelGGL((k_spmm<false, true>), g, b, 0, s, N, r0, c0, rp, ci, w, scale, in, out);
  else if (!acc) hipLaunchKernelGGL((k_spmm<true, false>), g, b, 0, s, N, r0, c0, rp, ci, w, scale, in, out);
  else hipLaunchKernelGGL((k_spmm<true, true>), g, b, 0, s, N, r0, c0, rp, ci, w, scale, in, out);
}
void launch_gemm_fwd(int N, const float* A0, const float* A1, const unsigned short* Wt, const float* bias, float* Y,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_gemm_fwd, dim3(grid_for(N, 64, 4096)), dim3(kBlock), 0, s, N, A0, A1, Wt, bias, Y);
}
void launch_head(int N, const float* H, const float* w, const float* b, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_head, dim3(grid_for((int64_t)N * kH)), dim3(kBlock), 0, s, N, H, w, b, out);
}
void launch_pool(int count, const int32_t* voff, const int32_t* coff, int v0, int c0, const float* Hv,
                 const float* Hc, const float* wo, const float* bo, float* pool, float* poolpart, float* oh,
                 hipStream_t s) {
  if (count <= 0) return;
  const int64_t tasks = (int64_t)count * kPoolSlices;
  hipLaunchKernelGGL(k_pool_part, dim3((unsigned)std::min<int64_t>(tasks, 16384)), dim3(kBlock), 0, s, count, voff,
                     coff, v0, c0, Hv, Hc, poolpart);
  hipLaunchKernelGGL(k_pool_fin, dim3((unsigned)std::min<int64_t>((count + kBlock / 64 - 1) / (kBlock / 64), 4096)), dim3(kBlock), 0, s, count,
                     voff, coff, poolpart, wo, bo, pool, oh);
}
void launch_loss(int count, int first, const int32_t* voff, const int32_t* coff, int v0, int c0, const float* xh,
                 const float* yh, const float* oh, const float* xt, const float* yt, const float* ot, float wx,
                 float wy, float wo, float* dxh, float* dyh, float* doh, double* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_loss, dim3(count < 8192 ? count : 8192), dim3(kBlock), 0, s, count, first, voff, coff, v0, c0,
                     xh, yh, oh, xt, yt, ot, wx, wy, wo, dxh, dyh, doh, loss);
}
void launch_predict(int nv, int nc, int v0, int c0, const int32_t* vown, const int32_t* cown, const double* scales,
                    const float* xh, const float* yh, double* x0, double* y0, hipStream_t s) {
  hipLaunchKernelGGL(k_predict, dim3(grid_for(nv > nc ? nv : nc)), dim3(kBlock), 0, s, nv, nc, v0, c0, vown, cown,
                     scales, xh, yh, x0, y0);
}
void launch_omega(int count, const float* oh, double* om, hipStream_t s) {
  hipLaunchKernelGGL(k_omega, dim3(grid_for(count)), dim3(kBlock), 0, s, count, oh, om);
}
int head_bwd_grid(int N) { return grid_for((int64_t)N * kH, kBlock, 1024); }
void launch_head_bwd(int N, int first, const int32_t* own, const int32_t* off, const float* H, const float* dh,
                     const float* doh, const float* w, const float* wo, float* dH, float* part, hipStream_t s) {
  hipLaunchKernelGGL(k_head_bwd, dim3(head_bwd_grid(N)), dim3(kBlock), 0, s, N, first, own, off, H, dh, doh, w, wo, dH,
                     part);
}
void launch_pool_bwd(int count, const float* pool, const float* doh, float* g, hipStream_t s) {
  hipLaunchKernelGGL(k_pool_bwd, dim3(1), dim3(192), 0, s, count, pool, doh, g);
}
void launch_gemm_dx(int N, const float* dH, const float* Hout, const unsigned short* Wb, float* D0, float* D1,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_gemm_dx, dim3(grid_for(N, 64, 4096)), dim3(kBlock), 0, s, N, dH, Hout, Wb, D0, D1);
}
// rows per workgroup of k_gemm_dw (a multiple of 32) and its grid
void dw_shape(int N, int* rows_per_wg, int* grid) {
  int g = 512;
  int r = (N + g - 1) / g;
  r = ((r + 31) / 32) * 32;
  if (r < 32) r = 32;
  *rows_per_wg = r;
  *grid = N > 0 ? (N + r - 1) / r : 1;
}
void launch_gemm_dw(int N, int rows_per_wg, int grid, const float* A0, const float* A1, const float* dH,
                    const float* Hout, float* part, hipStream_t s) {
  hipLaunchKernelGGL(k_gemm_dw, dim3(grid), dim3(kBlock), 0, s, N, rows_per_wg, A0, A1, dH, Hout, part);
}
int embed_bwd_grid(int N) { return grid_for((int64_t)N * kH, kBlock, 1024); }
void launch_embed_bwd(int N, int fdim, const float* F, const float* dH, const float* H, float* part, hipStream_t s) {
  hipLaunchKernelGGL(k_embed_bwd, dim3(embed_bwd_grid(N)), dim3(kBlock), 0, s, N, fdim, F, dH, H, part);
}
void launch_sum_parts(int nparts, int width, const float* part, float* g, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)std::max(1, (width + 63) / 64)), dim3(kBlock), 0, s, nparts, width,
                     part, g);
}
void launch_adam(int n, float* th, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(kBlock), 0, s, n, th, g, m, v, lr, b1, b2, eps, c1, c2);
}

}  // namespace gnnk
