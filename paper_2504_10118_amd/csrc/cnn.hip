// Learned-start kernels for gfx950: direct 3x3 convolutions staged through
// LDS (forward, backward-data via transposed weights, weight gradients with
// fixed-order partial sums), the complex MSE head, Adam, the network input
// map computed from the measured intensities, and whole-object
// restriction / prolongation (2x2 average pooling and 2x2 replication applied
// repeatedly, i.e. f x f block means and copies).
//
// All reductions run in a fixed order, so every result is bitwise
// reproducible run to run.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cnn.h"

namespace cnn {

namespace {

constexpr int CT = CONV_TILE;
constexpr int HALO = CT + 2;     // 18
constexpr int CCH = 8;           // input channels per LDS stage (forward)
constexpr int CPITCH = HALO + 1; // odd row pitch of the forward halo tile

__device__ __forceinline__ float wload(const float* w, size_t i) { return w[i]; }
__device__ __forceinline__ float wload(const uint16_t* w, size_t i) {
  return __uint_as_float((uint32_t)w[i] << 16);
}

__device__ __forceinline__ uint16_t to_bf16(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// ---------------------------------------------------------------------------
// Convolution (forward and backward-data)
// ---------------------------------------------------------------------------
template <int CO, bool UP, int MODE, typename WT>
__global__ __launch_bounds__(256) void conv3x3_kernel(const float* __restrict__ in, const WT* __restrict__ w,
                                                      const float* __restrict__ bias, float* __restrict__ out,
                                                      const float* __restrict__ omask, int ci_n, int H, int W) {
  __shared__ float tile[CCH][HALO][CPITCH];
  const int tx = threadIdx.x & (CT - 1), ty = threadIdx.x / CT;
  const int x0 = blockIdx.x * CT, y0 = blockIdx.y * CT, b = blockIdx.z;
  const int Hi = UP ? (H >> 1) : H, Wi = UP ? (W >> 1) : W;
  const float* inb = in + (size_t)b * ci_n * Hi * Wi;
  float acc[CO];
#pragma unroll
  for (int o = 0; o < CO; ++o) acc[o] = (MODE <= 1) ? bias[o] : 0.0f;
  for (int c0 = 0; c0 < ci_n; c0 += CCH) {
    const int nc = min(CCH, ci_n - c0);
    for (int i = threadIdx.x; i < nc * HALO * HALO; i += 256) {
      const int c = i / (HALO * HALO), r = i - c * HALO * HALO;
      const int yy = r / HALO, xx = r - yy * HALO;
      const int gy = y0 + yy - 1, gx = x0 + xx - 1;
      float v = 0.0f;
      if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
        const int sy = UP ? (gy >> 1) : gy, sx = UP ? (gx >> 1) : gx;
        v = inb[((size_t)(c0 + c) * Hi + sy) * Wi + sx];
      }
      tile[c][yy][xx] = v;
    }
    __syncthreads();
    for (int c = 0; c < nc; ++c) {
      float xv[9];
#pragma unroll
      for (int t = 0; t < 9; ++t) xv[t] = tile[c][ty + t / 3][tx + t % 3];
      const size_t wb = (size_t)(c0 + c) * 9;
#pragma unroll
      for (int o = 0; o < CO; ++o) {
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[o] = fmaf(wload(w, wb + (size_t)o * ci_n * 9 + t), xv[t], acc[o]);
      }
    }
    __syncthreads();
  }
  const int oy = y0 + ty, ox = x0 + tx;
  if (oy < H && ox < W) {
    const size_t plane = (size_t)H * W;
    const size_t base = (size_t)b * CO * plane + (size_t)oy * W + ox;
#pragma unroll
    for (int o = 0; o < CO; ++o) {
      float v = acc[o];
      if (MODE == 0) v = fmaxf(v, 0.0f);
      if (MODE == 2) v = (omask[base + o * plane] > 0.0f) ? v : 0.0f;
      out[base + o * plane] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Weight gradients: each workgroup walks a contiguous run of 16x16 output
// tiles; thread (cog, c) owns output channels 4*cog .. 4*cog+3 and input
// channel c, i.e. 36 weight sums and 4 bias sums.
// ---------------------------------------------------------------------------
constexpr int WG_TILES_TARGET = WGRAD_MAX_WORKGROUPS;
constexpr int IN_PITCH = HALO * HALO + 1;  // 325: odd, so the 32 input channels hit 32 banks
constexpr int DO_PITCH = CT * CT + 1;      // 257

template <bool UP>
__global__ __launch_bounds__(256) void wgrad_kernel(const float* __restrict__ in, const float* __restrict__ dout,
                                                    float* __restrict__ part, int ci_n, int co_n, int H, int W,
                                                    int tiles_x, int tiles_per_sample, int total_tiles,
                                                    int tiles_per_wg) {
  __shared__ float sin_[MAX_WIDTH * IN_PITCH];
  __shared__ float sdo[MAX_WIDTH * DO_PITCH];
  const int c = threadIdx.x & 31, cog = threadIdx.x >> 5;
  const bool active = c < ci_n && cog * 4 < co_n;
  const int Hi = UP ? (H >> 1) : H, Wi = UP ? (W >> 1) : W;
  float acc[4][9];
  float bacc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    bacc[j] = 0.0f;
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[j][t] = 0.0f;
  }
  const int t_begin = blockIdx.x * tiles_per_wg;
  const int t_end = min(total_tiles, t_begin + tiles_per_wg);
  for (int tile = t_begin; tile < t_end; ++tile) {
    const int b = tile / tiles_per_sample, tr = tile - b * tiles_per_sample;
    const int y0 = (tr / tiles_x) * CT, x0 = (tr % tiles_x) * CT;
    const float* inb = in + (size_t)b * ci_n * Hi * Wi;
    const float* dob = dout + (size_t)b * co_n * H * W;
    for (int i = threadIdx.x; i < ci_n * HALO * HALO; i += 256) {
      const int cc = i / (HALO * HALO), r = i - cc * HALO * HALO;
      const int yy = r / HALO, xx = r - yy * HALO;
      const int gy = y0 + yy - 1, gx = x0 + xx - 1;
      float v = 0.0f;
      if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
        const int sy = UP ? (gy >> 1) : gy, sx = UP ? (gx >> 1) : gx;
        v = inb[((size_t)cc * Hi + sy) * Wi + sx];
      }
      sin_[cc * IN_PITCH + r] = v;
    }
    for (int i = threadIdx.x; i < co_n * CT * CT; i += 256) {
      const int o = i / (CT * CT), p = i - o * CT * CT;
      const int gy = y0 + p / CT, gx = x0 + p % CT;
      sdo[o * DO_PITCH + p] = (gy < H && gx < W) ? dob[((size_t)o * H + gy) * W + gx] : 0.0f;
    }
    __syncthreads();
    if (active) {
      for (int p = 0; p < CT * CT; ++p) {
        const int py = p / CT, px = p % CT;
        float g[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) g[j] = (cog * 4 + j < co_n) ? sdo[(cog * 4 + j) * DO_PITCH + p] : 0.0f;
        float xv[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) xv[t] = sin_[c * IN_PITCH + (py + t / 3) * HALO + px + t % 3];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          bacc[j] += g[j];
#pragma unroll
          for (int t = 0; t < 9; ++t) acc[j][t] = fmaf(g[j], xv[t], acc[j][t]);
        }
      }
    }
    __syncthreads();
  }
  if (!active) return;
  const size_t row = (size_t)co_n * ci_n * 9 + co_n;
  float* pr = part + (size_t)blockIdx.x * row;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int o = cog * 4 + j;
    if (o >= co_n) break;
#pragma unroll
    for (int t = 0; t < 9; ++t) pr[((size_t)o * ci_n + c) * 9 + t] = acc[j][t];
    if (c == 0) pr[(size_t)co_n * ci_n * 9 + o] = bacc[j];
  }
}

// grad[j] = sum_r part[r][j]: 64 columns per block, 4 strided row sets combined in order.
__global__ __launch_bounds__(256) void rows_sum_kernel(const float* __restrict__ part, int n_rows, int row_len,
                                                       float* __restrict__ grad) {
  __shared__ float red[4][64];
  const int jj = threadIdx.x & 63, s = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + jj;
  float acc = 0.0f;
  if (j < row_len)
    for (int r = s; r < n_rows; r += 4) acc += part[(size_t)r * row_len + j];
  red[s][jj] = acc;
  __syncthreads();
  if (s == 0 && j < row_len) grad[j] = ((red[0][jj] + red[1][jj]) + red[2][jj]) + red[3][jj];
}

__global__ void up_backward_mask_kernel(const float* __restrict__ du, const float* __restrict__ a,
                                        float* __restrict__ da, size_t total, int H, int W) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const size_t bc = i / ((size_t)H * W);
  const int r = (int)(i - bc * H * W);
  const int y = r / W, x = r - y * W;
  const float* src = du + bc * (size_t)(4 * H * W) + (size_t)(2 * y) * (2 * W) + 2 * x;
  const float sum = (src[0] + src[1]) + (src[2 * W] + src[2 * W + 1]);
  da[i] = (a[i] > 0.0f) ? sum : 0.0f;
}

// ---------------------------------------------------------------------------
// Complex MSE head
// ---------------------------------------------------------------------------
constexpr int CMSE_THREADS = 256;

__device__ __forceinline__ float2 pred_of(const float* __restrict__ y, size_t b, int p, int hw) {
  const float la = y[(b * 2) * hw + p], ph = y[(b * 2 + 1) * hw + p];
  float sn, cs;
  sincosf(ph, &sn, &cs);
  const float amp = expf(la);
  return make_float2(amp * cs, amp * sn);
}

// per-block partial sums of mask * conj(pred) * t for each sample: part[b][blockIdx.x]
__global__ __launch_bounds__(CMSE_THREADS) void cmse_ip_kernel(const float* __restrict__ y,
                                                               const float2* __restrict__ tgt,
                                                               const float* __restrict__ mask,
                                                               double2* __restrict__ part, int hw) {
  __shared__ double rr[CMSE_THREADS], ri[CMSE_THREADS];
  const int b = blockIdx.y;
  const int p = blockIdx.x * CMSE_THREADS + threadIdx.x;
  double a = 0.0, c = 0.0;
  if (p < hw) {
    const float2 pr = pred_of(y, b, p, hw);
    const float2 t = tgt[(size_t)b * hw + p];
    const double mk = mask[p];
    a = mk * ((double)pr.x * t.x + (double)pr.y * t.y);
    c = mk * ((double)pr.x * t.y - (double)pr.y * t.x);
  }
  rr[threadIdx.x] = a;
  ri[threadIdx.x] = c;
  __syncthreads();
  for (int s = CMSE_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      rr[threadIdx.x] += rr[threadIdx.x + s];
      ri[threadIdx.x] += ri[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)b * gridDim.x + blockIdx.x] = make_double2(rr[0], ri[0]);
}

// rot[b] = ip / |ip| (1 where ip = 0), ip = sum of the sample's partials in order
__global__ __launch_bounds__(256) void cmse_rot_kernel(const double2* __restrict__ part, int nblk,
                                                       float2* __restrict__ rot) {
  __shared__ double rr[256], ri[256];
  const int b = blockIdx.x;
  double a = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < nblk; i += 256) {
    a += part[(size_t)b * nblk + i].x;
    c += part[(size_t)b * nblk + i].y;
  }
  rr[threadIdx.x] = a;
  ri[threadIdx.x] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      rr[threadIdx.x] += rr[threadIdx.x + s];
      ri[threadIdx.x] += ri[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double n = sqrt(rr[0] * rr[0] + ri[0] * ri[0]);
    rot[b] = n > 0.0 ? make_float2((float)(rr[0] / n), (float)(ri[0] / n)) : make_float2(1.0f, 0.0f);
  }
}

__global__ __launch_bounds__(CMSE_THREADS) void cmse_kernel(const float* __restrict__ y,
                                                            const float2* __restrict__ tgt,
                                                            const float* __restrict__ mask,
                                                            const float2* __restrict__ rot, float* __restrict__ dy,
                                                            double* __restrict__ part, int batch, int hw,
                                                            float inv_norm) {
  __shared__ double red[CMSE_THREADS];
  const size_t i = (size_t)blockIdx.x * CMSE_THREADS + threadIdx.x;
  double l = 0.0;
  if (i < (size_t)batch * hw) {
    const size_t b = i / hw;
    const int p = (int)(i - b * hw);
    float2 pv = pred_of(y, b, p, hw);
    if (rot) {
      const float2 r = rot[b];
      pv = make_float2(pv.x * r.x - pv.y * r.y, pv.x * r.y + pv.y * r.x);
    }
    const float pr = pv.x, pi = pv.y;
    const float2 t = tgt[i];
    const float rr = pr - t.x, ri = pi - t.y;
    const float mk = mask[p];
    l = (double)mk * ((double)rr * rr + (double)ri * ri);
    // g = conj(r) * pred
    const float gr = rr * pr + ri * pi, gi = rr * pi - ri * pr;
    dy[(b * 2) * hw + p] = 2.0f * mk * gr * inv_norm;
    dy[(b * 2 + 1) * hw + p] = -2.0f * mk * gi * inv_norm;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = CMSE_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void sum_f64_kernel(const double* __restrict__ x, int n, double* __restrict__ out) {
  __shared__ double red[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) a += x[i];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// ---------------------------------------------------------------------------
// Adam and weight copies
// ---------------------------------------------------------------------------
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

template <typename WT>
__device__ __forceinline__ WT cvt_w(float x);
template <>
__device__ __forceinline__ float cvt_w<float>(float x) { return x; }
template <>
__device__ __forceinline__ uint16_t cvt_w<uint16_t>(float x) { return to_bf16(x); }

template <typename WT>
__global__ void prep_weights_kernel(const float* __restrict__ p, WT* __restrict__ wf, WT* __restrict__ wt, int co,
                                    int ci) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= co * ci * 9) return;
  const int o = i / (ci * 9), r = i - o * ci * 9, c = r / 9, t = r - c * 9;
  const WT v = cvt_w<WT>(p[i]);
  wf[i] = v;
  wt[((size_t)c * co + o) * 9 + (8 - t)] = v;
}

// ---------------------------------------------------------------------------
// Network input map
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void probe_norm_kernel(const double2* __restrict__ q, int mm,
                                                         double* __restrict__ out) {
  __shared__ double red[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < mm; i += 256) a += q[i].x * q[i].x + q[i].y * q[i].y;
  red[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(red[0]);
}

__global__ __launch_bounds__(256) void position_stats_kernel(const float* __restrict__ sqrtd, int m,
                                                             const double* __restrict__ qnorm,
                                                             double4* __restrict__ stats) {
  __shared__ double red[4][256];
  const int k = blockIdx.x;
  const float* s = sqrtd + (size_t)k * m * m;
  double sa = 0.0, sd = 0.0, sy = 0.0, sx = 0.0;
  for (int i = threadIdx.x; i < m * m; i += 256) {
    const int r = i / m, c = i - r * m;
    const double a = (double)s[i];
    const double d = a * a;
    const double fy = (r < m / 2) ? r : r - m, fx = (c < m / 2) ? c : c - m;
    sa += a;
    sd += d;
    sy += fy * d;
    sx += fx * d;
  }
  red[0][threadIdx.x] = sa;
  red[1][threadIdx.x] = sd;
  red[2][threadIdx.x] = sy;
  red[3][threadIdx.x] = sx;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st)
#pragma unroll
      for (int j = 0; j < 4; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double tot = red[1][0];
    double4 o;
    o.x = red[0][0] / ((double)m * m) / qnorm[0];
    o.y = tot > 0.0 ? red[2][0] / tot : 0.0;
    o.z = tot > 0.0 ? red[3][0] / tot : 0.0;
    o.w = 0.0;
    stats[k] = o;
  }
}

__global__ void map_fine_kernel(const double4* __restrict__ stats, const double2* __restrict__ q, int m,
                                const int* __restrict__ tile_ptr, const int4* __restrict__ tile_ent, int tiles_x,
                                int tile_w, int tile_h, int nr, int nc, double* __restrict__ fine) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (c >= nc) return;
  const int t = (r / tile_h) * tiles_x + c / tile_w;
  double n0 = 0.0, n1 = 0.0, n2 = 0.0, den = 0.0;
  for (int e = tile_ptr[t]; e < tile_ptr[t + 1]; ++e) {
    const int4 en = tile_ent[e];
    const int dr = r - en.y, dc = c - en.z;
    if (dr < 0 || dr >= m || dc < 0 || dc >= m) continue;
    const double2 qv = q[dr * m + dc];
    const double w = qv.x * qv.x + qv.y * qv.y;
    const double4 s = stats[en.x];
    n0 += w * s.x;
    n1 += w * s.y;
    n2 += w * s.z;
    den += w;
  }
  const size_t plane = (size_t)nr * nc, i = (size_t)r * nc + c;
  const bool pos = den > 0.0;
  fine[i] = pos ? n0 / den : 0.0;
  fine[plane + i] = pos ? n1 / den : 0.0;
  fine[2 * plane + i] = pos ? n2 / den : 0.0;
}

__global__ void pool_kernel(const double* __restrict__ fine, int nr, int nc, int fr, int fc, float* __restrict__ out) {
  const int so = nc / fc, sr = nr / fr;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y, ch = blockIdx.z;
  if (j >= so || i >= sr) return;
  const double* src = fine + (size_t)ch * nr * nc;
  double a = 0.0;
  for (int y = 0; y < fr; ++y)
    for (int x = 0; x < fc; ++x) a += src[(size_t)(i * fr + y) * nc + j * fc + x];
  out[((size_t)ch * sr + i) * so + j] = (float)(a / ((double)fr * fc));
}

// Phase channel: least-squares integration of the gradient field the two
// centre-of-mass channels measure (Frankot and Chellappa), in FP64 on one
// workgroup.  The two real fields are transformed together as
// H = DFT(gy + i gx) and separated with the conjugate-symmetric parts; then
// phi^ = -i (wy Gy + wx Gx) / (wy^2 + wx^2) (0 at zero frequency) and
// phi = Re IDFT(phi^).  Direct DFT sums over rows and columns (S <= 64).
constexpr int PHI_MAX_S = 64;
constexpr int PHI_THREADS = 1024;

__global__ __launch_bounds__(PHI_THREADS) void integrate_phase_kernel(const float* __restrict__ gy_in,
                                                                      const float* __restrict__ gx_in, int S,
                                                                      double sy, double sx,
                                                                      float* __restrict__ out) {
  __shared__ double2 A[PHI_MAX_S * PHI_MAX_S];
  __shared__ double2 Bf[PHI_MAX_S * PHI_MAX_S];
  __shared__ double2 W[PHI_MAX_S];
  const int tid = threadIdx.x, SS = S * S;
  for (int j = tid; j < S; j += PHI_THREADS) {
    double sn, cs;
    sincospi(-2.0 * j / S, &sn, &cs);
    W[j] = make_double2(cs, sn);   // exp(-2 pi i j / S)
  }
  for (int e = tid; e < SS; e += PHI_THREADS) A[e] = make_double2(sy * gy_in[e], sx * gx_in[e]);
  __syncthreads();
  // forward: rows, then columns
  for (int e = tid; e < SS; e += PHI_THREADS) {
    const int y = e / S, k = e - y * S;
    double2 acc = make_double2(0.0, 0.0);
    for (int x = 0; x < S; ++x) {
      const double2 a = A[y * S + x], w = W[(k * x) % S];
      acc.x += a.x * w.x - a.y * w.y;
      acc.y += a.x * w.y + a.y * w.x;
    }
    Bf[e] = acc;
  }
  __syncthreads();
  for (int e = tid; e < SS; e += PHI_THREADS) {
    const int k0 = e / S, k1 = e - k0 * S;
    double2 acc = make_double2(0.0, 0.0);
    for (int y = 0; y < S; ++y) {
      const double2 b = Bf[y * S + k1], w = W[(k0 * y) % S];
      acc.x += b.x * w.x - b.y * w.y;
      acc.y += b.x * w.y + b.y * w.x;
    }
    A[e] = acc;
  }
  __syncthreads();
  // separate the two spectra, divide by |w|^2
  for (int e = tid; e < SS; e += PHI_THREADS) {
    const int k0 = e / S, k1 = e - k0 * S;
    const int m0 = (S - k0) % S, m1 = (S - k1) % S;
    const double2 h = A[e], hm = A[m0 * S + m1];
    // Gy = (h + conj(hm)) / 2, Gx = (h - conj(hm)) / (2 i)
    const double2 gy = make_double2(0.5 * (h.x + hm.x), 0.5 * (h.y - hm.y));
    const double2 gx = make_double2(0.5 * (h.y + hm.y), -0.5 * (h.x - hm.x));
    const int f0 = (k0 < (S + 1) / 2) ? k0 : k0 - S, f1 = (k1 < (S + 1) / 2) ? k1 : k1 - S;
    const double wy = 6.283185307179586 * f0 / S, wx = 6.283185307179586 * f1 / S;
    const double den = wy * wy + wx * wx;
    double2 ph = make_double2(0.0, 0.0);
    if (den > 0.0) {
      // -i (wy gy + wx gx) / den
      const double2 t = make_double2(wy * gy.x + wx * gx.x, wy * gy.y + wx * gx.y);
      ph = make_double2(t.y / den, -t.x / den);
    }
    Bf[e] = ph;
  }
  __syncthreads();
  // inverse: columns, then rows; real part / S^2
  for (int e = tid; e < SS; e += PHI_THREADS) {
    const int y = e / S, k1 = e - y * S;
    double2 acc = make_double2(0.0, 0.0);
    for (int k0 = 0; k0 < S; ++k0) {
      const double2 b = Bf[k0 * S + k1], w = W[(k0 * y) % S];
      acc.x += b.x * w.x + b.y * w.y;    // times conj(w)
      acc.y += b.y * w.x - b.x * w.y;
    }
    A[e] = acc;
  }
  __syncthreads();
  for (int e = tid; e < SS; e += PHI_THREADS) {
    const int y = e / S, x = e - y * S;
    double acc = 0.0;
    for (int k1 = 0; k1 < S; ++k1) {
      const double2 a = A[y * S + k1], w = W[(k1 * x) % S];
      acc += a.x * w.x + a.y * w.y;      // Re(a conj(w))
    }
    out[e] = (float)(acc / ((double)S * S));
  }
}

// ---------------------------------------------------------------------------
// Whole-object prolongation and restriction
// ---------------------------------------------------------------------------
__global__ void prolong_object_kernel(const void* __restrict__ coarse, int format, int sr, int sc, int f,
                                      float2* __restrict__ z, int nr, int nc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (c >= nc) return;
  const int i = r / f, j = c / f;
  const size_t ci = (size_t)i * sc + j;
  float2 v;
  if (format == 0) {
    v = ((const float2*)coarse)[ci];
  } else if (format == 1) {
    const double2 d = ((const double2*)coarse)[ci];
    v = make_float2((float)d.x, (float)d.y);
  } else {
    const float* pl = (const float*)coarse;
    const float amp = expf(pl[ci]);
    float sn, cs;
    sincosf(pl[(size_t)sr * sc + ci], &sn, &cs);
    v = make_float2(amp * cs, amp * sn);
  }
  z[(size_t)r * nc + c] = v;
}

__global__ void restrict_object_kernel(const float2* __restrict__ z, int nr, int nc, int f, float2* __restrict__ out) {
  const int so = nc / f, sr = nr / f;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= so || i >= sr) return;
  double ax = 0.0, ay = 0.0;
  for (int y = 0; y < f; ++y)
    for (int x = 0; x < f; ++x) {
      const float2 v = z[(size_t)(i * f + y) * nc + j * f + x];
      ax += v.x;
      ay += v.y;
    }
  const double inv = 1.0 / ((double)f * f);
  out[(size_t)i * so + j] = make_float2((float)(ax * inv), (float)(ay * inv));
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <int CO, bool UP, int MODE>
static void conv_t(bool bf16, const float* in, const void* w, const float* bias, float* out, const float* omask,
                   int batch, int ci, int H, int W, hipStream_t s) {
  const dim3 grid((W + CT - 1) / CT, (H + CT - 1) / CT, batch);
  if (bf16)
    hipLaunchKernelGGL((conv3x3_kernel<CO, UP, MODE, uint16_t>), grid, dim3(256), 0, s, in, (const uint16_t*)w, bias,
                       out, omask, ci, H, W);
  else
    hipLaunchKernelGGL((conv3x3_kernel<CO, UP, MODE, float>), grid, dim3(256), 0, s, in, (const float*)w, bias, out,
                       omask, ci, H, W);
}

hipError_t launch_conv(int co, bool up, int mode, bool bf16, const float* in, const void* w, const float* bias,
                       float* out, const float* omask, int batch, int ci, int H, int W, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  if (ci < 1 || H < 1 || W < 1 || (up && ((H | W) & 1))) return hipErrorInvalidValue;
#define CNN_CONV(CO_, UP_, MODE_)                                                                  \
  if (co == CO_ && up == UP_ && mode == MODE_) {                                                   \
    conv_t<CO_, UP_, MODE_>(bf16, in, w, bias, out, omask, batch, ci, H, W, s);                    \
    return hipGetLastError();                                                                      \
  }
  // forward: 0 (ReLU) for the hidden layers, 1 (linear) for the head; backward-data: 2 (masked), 3
  CNN_CONV(32, false, 0)
  CNN_CONV(32, true, 0)
  CNN_CONV(2, false, 1)
  CNN_CONV(32, false, 2)
  CNN_CONV(32, false, 3)
#undef CNN_CONV
  return hipErrorInvalidValue;
}

int wgrad_workgroups(int batch, int H, int W) {
  const int tiles = batch * ((H + CT - 1) / CT) * ((W + CT - 1) / CT);
  const int per = (tiles + WG_TILES_TARGET - 1) / WG_TILES_TARGET;
  return (tiles + per - 1) / per;
}

hipError_t launch_wgrad(bool up, const float* in, const float* dout, float* part, int batch, int ci, int co, int H,
                        int W, hipStream_t s) {
  if (batch <= 0) return hipSuccess;
  if (ci < 1 || ci > MAX_WIDTH || co < 1 || co > MAX_WIDTH || (up && ((H | W) & 1))) return hipErrorInvalidValue;
  const int tiles_x = (W + CT - 1) / CT;
  const int per_sample = tiles_x * ((H + CT - 1) / CT);
  const int tiles = batch * per_sample;
  const int per = (tiles + WG_TILES_TARGET - 1) / WG_TILES_TARGET;
  const int nwg = (tiles + per - 1) / per;
  if (up)
    hipLaunchKernelGGL(wgrad_kernel<true>, dim3(nwg), dim3(256), 0, s, in, dout, part, ci, co, H, W, tiles_x,
                       per_sample, tiles, per);
  else
    hipLaunchKernelGGL(wgrad_kernel<false>, dim3(nwg), dim3(256), 0, s, in, dout, part, ci, co, H, W, tiles_x,
                       per_sample, tiles, per);
  return hipGetLastError();
}

hipError_t launch_rows_sum(const float* part, int n_rows, int row_len, float* grad, hipStream_t s) {
  if (row_len <= 0) return hipSuccess;
  hipLaunchKernelGGL(rows_sum_kernel, dim3((row_len + 63) / 64), dim3(256), 0, s, part, n_rows, row_len, grad);
  return hipGetLastError();
}

hipError_t launch_up_backward_mask(const float* du, const float* a, float* da, int batch, int C, int H, int W,
                                   hipStream_t s) {
  const size_t total = (size_t)batch * C * H * W;
  if (!total) return hipSuccess;
  hipLaunchKernelGGL(up_backward_mask_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, du, a, da,
                     total, H, W);
  return hipGetLastError();
}

int cmse_blocks(int batch, int hw) { return (int)(((size_t)batch * hw + CMSE_THREADS - 1) / CMSE_THREADS); }

int cmse_ip_blocks(int hw) { return (hw + CMSE_THREADS - 1) / CMSE_THREADS; }

hipError_t launch_cmse(const float* y, const float2* target, const float* mask, float2* rot, double2* ip_part,
                       float* dy, double* part, int batch, int hw, float inv_norm, hipStream_t s) {
  const int nb = cmse_blocks(batch, hw);
  if (nb <= 0) return hipSuccess;
  if (rot) {
    const int nbi = cmse_ip_blocks(hw);
    hipLaunchKernelGGL(cmse_ip_kernel, dim3(nbi, batch), dim3(CMSE_THREADS), 0, s, y, target, mask, ip_part, hw);
    hipLaunchKernelGGL(cmse_rot_kernel, dim3(batch), dim3(256), 0, s, ip_part, nbi, rot);
  }
  hipLaunchKernelGGL(cmse_kernel, dim3(nb), dim3(CMSE_THREADS), 0, s, y, target, mask, (const float2*)rot, dy, part,
                     batch, hw, inv_norm);
  return hipGetLastError();
}

hipError_t launch_sum_f64(const double* x, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sum_f64_kernel, dim3(1), dim3(256), 0, s, x, n, out);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps,
                     c1, c2);
  return hipGetLastError();
}

hipError_t launch_prep_weights(const float* p, void* wf, void* wt, int co, int ci, bool bf16, hipStream_t s) {
  const int n = co * ci * 9;
  if (bf16)
    hipLaunchKernelGGL(prep_weights_kernel<uint16_t>, dim3((n + 255) / 256), dim3(256), 0, s, p, (uint16_t*)wf,
                       (uint16_t*)wt, co, ci);
  else
    hipLaunchKernelGGL(prep_weights_kernel<float>, dim3((n + 255) / 256), dim3(256), 0, s, p, (float*)wf, (float*)wt,
                       co, ci);
  return hipGetLastError();
}

hipError_t launch_probe_norm(const double2* q, int m, double* out, hipStream_t s) {
  hipLaunchKernelGGL(probe_norm_kernel, dim3(1), dim3(256), 0, s, q, m * m, out);
  return hipGetLastError();
}

hipError_t launch_position_stats(const float* sqrtd, int n_pos, int m, const double* qnorm, double4* stats,
                                 hipStream_t s) {
  if (n_pos <= 0) return hipSuccess;
  hipLaunchKernelGGL(position_stats_kernel, dim3(n_pos), dim3(256), 0, s, sqrtd, m, qnorm, stats);
  return hipGetLastError();
}

hipError_t launch_map_fine(const double4* stats, const double2* q, int m, const int* tile_ptr, const int4* tile_ent,
                           int tiles_x, int tile_w, int tile_h, int nr, int nc, double* fine, hipStream_t s) {
  hipLaunchKernelGGL(map_fine_kernel, dim3((nc + 255) / 256, nr), dim3(256), 0, s, stats, q, m, tile_ptr, tile_ent,
                     tiles_x, tile_w, tile_h, nr, nc, fine);
  return hipGetLastError();
}

hipError_t launch_pool(const double* fine, int nr, int nc, int fr, int fc, float* out, hipStream_t s) {
  const int so = nc / fc, sr = nr / fr;
  hipLaunchKernelGGL(pool_kernel, dim3((so + 63) / 64, sr, 3), dim3(64), 0, s, fine, nr, nc, fr, fc, out);
  return hipGetLastError();
}

hipError_t launch_integrate_phase(const float* gy, const float* gx, int S, double sy, double sx, float* out,
                                  hipStream_t s) {
  if (S < 1 || S > PHI_MAX_S) return hipErrorInvalidValue;
  hipLaunchKernelGGL(integrate_phase_kernel, dim3(1), dim3(PHI_THREADS), 0, s, gy, gx, S, sy, sx, out);
  return hipGetLastError();
}

hipError_t launch_prolong_object(const void* coarse, int format, int sr, int sc, int f, float2* z, int nr, int nc,
                                 hipStream_t s) {
  hipLaunchKernelGGL(prolong_object_kernel, dim3((nc + 255) / 256, nr), dim3(256), 0, s, coarse, format, sr, sc, f, z,
                     nr, nc);
  return hipGetLastError();
}

hipError_t launch_restrict_object(const float2* z, int nr, int nc, int f, float2* out, hipStream_t s) {
  const int so = nc / f, sr = nr / f;
  hipLaunchKernelGGL(restrict_object_kernel, dim3((so + 63) / 64, sr), dim3(64), 0, s, z, nr, nc, f, out);
  return hipGetLastError();
}

}  // namespace cnn
