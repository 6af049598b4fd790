// gfx950 kernels of the MAGPIE hot path (arXiv 2504.10118).
//
// step_kernel<M, MODE>  one workgroup per scan position: gather z_k, exit wave
//                       Q * z_k, LDS-resident 2-D FFT, modulus replacement
//                       (Definition 2.1), inverse FFT, gradient
//                       g0 = conj(Q)(Q z_k - R_k) (eq. 2.2), MAGPS V-cycle in
//                       gradient form (Alg 3 / eq. 4.6), write c_k = w0 * dz_k.
// accumulate_kernel     one workgroup per 64 x 16 object tile: fixed-order sum
//                       of the overlapping c_k and of w0 (FP64), z += N / D.
// level_constants_kernel FP64 probe hierarchy (eq. 4.4) and per-level
//                       coefficients of the gradient-form V-cycle.
//
// 2-D FFT layout.  M = RA * RB.  A workgroup has M * RB threads; thread
// tid = lo + M * g (lo in [0, M), g in [0, RB)).  Each 1-D pass along an axis
// is two register stages: stage A, a radix-RA DFT over elements RB apart,
// then the twiddle W_M^(n2 k1); stage B, CB = RA / RB radix-RB DFTs.  Data
// move between stages through one padded LDS tile [M][M + 1] of float2.
// Columns are transformed first with lo = x (lanes read whole object rows);
// rows second with lo = ky.  The forward output lands with thread (ky, g)
// holding kx = g*CB + c + RA*k2, which is the order sqrt(d) is stored in, so
// the irreducible sqrt(d) stream is read as contiguous per-thread vectors.
// The inverse transform retraces the forward steps backwards and returns the
// data to the gather layout (thread (x, g) holds rows y = RB*n1 + g).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cmath.h"
#include "kernels.h"

namespace mg {

// W_128^j = exp(-2 pi i j / 128), j in [0, 128); filled once per device.
__device__ float2 g_twiddle[128];

__global__ void twiddle_init_kernel() {
  int j = threadIdx.x;
  if (j < 128) {
    double s, c;
    sincospi(-2.0 * j / 128.0, &s, &c);
    g_twiddle[j] = make_float2((float)c, (float)s);
  }
}

hipError_t init_twiddles(hipStream_t s) {
  hipLaunchKernelGGL(twiddle_init_kernel, dim3(1), dim3(128), 0, s);
  return hipGetLastError();
}

template <int M> struct Plan;
template <> struct Plan<8>   { static constexpr int RB = 2, RA = 4; };
template <> struct Plan<16>  { static constexpr int RB = 4, RA = 4; };
template <> struct Plan<32>  { static constexpr int RB = 4, RA = 8; };
template <> struct Plan<64>  { static constexpr int RB = 8, RA = 8; };
template <> struct Plan<128> { static constexpr int RB = 8, RA = 16; };

template <int M>
__device__ __forceinline__ float2 twiddle(int j) {
  return g_twiddle[(j & (M - 1)) * (128 / M)];
}

// Sum over the workgroup, fixed reduction order (deterministic).
template <int TPB>
__device__ __forceinline__ double block_sum(double v, double* red) {
  constexpr int W = TPB < 64 ? TPB : 64;
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, W);
  if constexpr (TPB <= 64) {
    return v;
  } else {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
      for (int w = 0; w < TPB / 64; ++w) s += red[w];
    }
    return s;
  }
}

template <int M, int MODE>
__global__ __launch_bounds__(M * Plan<M>::RB) void step_kernel(StepArgs a) {
  constexpr int RB = Plan<M>::RB, RA = Plan<M>::RA;
  constexpr int TPB = M * RB, CB = RA / RB, P = M + 1;
  extern __shared__ double2 smem_d2[];
  float2* buf = reinterpret_cast<float2*>(smem_d2);
  __shared__ double red[16];

  const int tid = threadIdx.x;
  const int lo = tid & (M - 1);
  int g = tid / M;
  if constexpr (M >= 64) g = __builtin_amdgcn_readfirstlane(g);
  const int k = a.perm ? a.perm[blockIdx.x] : (int)blockIdx.x;
  const int2 off = a.offs[k];

  // ---- gather z_k and form the exit wave Q * z_k (layout: thread (x=lo, g), rows RB*n1+g)
  float2 v[RA];
  const float2* zp = a.z + (size_t)off.x * a.n_cols + off.y + lo;
#pragma unroll
  for (int n1 = 0; n1 < RA; ++n1) {
    const int y = RB * n1 + g;
    v[n1] = cmul(a.q[y * M + lo], zp[(size_t)y * a.n_cols]);
  }
  // prefetch this thread's sqrt(d) values (contiguous RA floats)
  float sd[RA];
  if constexpr (MODE != MODE_FORWARD) {
    const float4* sp = reinterpret_cast<const float4*>(a.sqrtd + (size_t)k * M * M + (size_t)tid * RA);
#pragma unroll
    for (int i = 0; i < RA / 4; ++i) {
      float4 t = sp[i];
      sd[4 * i] = t.x; sd[4 * i + 1] = t.y; sd[4 * i + 2] = t.z; sd[4 * i + 3] = t.w;
    }
  }

  // ---- forward, columns (along y), stage A
  dft<RA, 1>(v);
#pragma unroll
  for (int k1 = 1; k1 < RA; ++k1) v[k1] = cmul(v[k1], twiddle<M>(g * k1));
#pragma unroll
  for (int k1 = 0; k1 < RA; ++k1) buf[(k1 * RB + g) * P + lo] = v[k1];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < CB; ++c)
#pragma unroll
    for (int n2 = 0; n2 < RB; ++n2) v[c * RB + n2] = buf[((g * CB + c) * RB + n2) * P + lo];
  // stage B
#pragma unroll
  for (int c = 0; c < CB; ++c) dft<RB, 1>(&v[c * RB]);
  __syncthreads();
  // transpose: buf[ky][x]
#pragma unroll
  for (int c = 0; c < CB; ++c)
#pragma unroll
    for (int k2 = 0; k2 < RB; ++k2) buf[((g * CB + c) + RA * k2) * P + lo] = v[c * RB + k2];
  __syncthreads();
  // ---- forward, rows (along x), stage A; lo = ky now
#pragma unroll
  for (int n1 = 0; n1 < RA; ++n1) v[n1] = buf[lo * P + RB * n1 + g];
  dft<RA, 1>(v);
#pragma unroll
  for (int k1 = 1; k1 < RA; ++k1) v[k1] = cmul(v[k1], twiddle<M>(g * k1));
  __syncthreads();
#pragma unroll
  for (int k1 = 0; k1 < RA; ++k1) buf[lo * P + k1 * RB + g] = v[k1];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < CB; ++c)
#pragma unroll
    for (int n2 = 0; n2 < RB; ++n2) v[c * RB + n2] = buf[lo * P + (g * CB + c) * RB + n2];
#pragma unroll
  for (int c = 0; c < CB; ++c) dft<RB, 1>(&v[c * RB]);
  // v[c*RB + k2] = Psi[ky = lo][kx = g*CB + c + RA*k2]

  if constexpr (MODE == MODE_FORWARD) {
    float* dp = a.d_out + (size_t)k * M * M + (size_t)lo * M;
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int k2 = 0; k2 < RB; ++k2) {
        float2 t = v[c * RB + k2];
        dp[g * CB + c + RA * k2] = t.x * t.x + t.y * t.y;
      }
    return;
  } else {
    // ---- modulus replacement (Definition 2.1, theta(0) = 0) and Phi_k partial (FP64)
    double phis = 0.0;
#pragma unroll
    for (int j = 0; j < RA; ++j) {
      const float2 t = v[j];
      const float a2 = t.x * t.x + t.y * t.y;
      const float am = sqrtf(a2);
      const float s = sd[j];
      const double dlt = (double)am - (double)s;
      phis += dlt * dlt;
      if (a2 > 0.0f) {
        const float f = s / am;
        v[j] = make_float2(t.x * f, t.y * f);
      } else {
        v[j] = make_float2(s, 0.0f);
      }
    }
    if (a.phi_k) {
      double tot = block_sum<TPB>(phis, red);
      if (tid == 0) a.phi_k[k] = tot * (0.5 / ((double)M * (double)M));
    }

    // ---- inverse, rows: stage B^-1, twiddle conj, stage A^-1
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      dft<RB, -1>(&v[c * RB]);
      const int k1 = g * CB + c;
#pragma unroll
      for (int n2 = 1; n2 < RB; ++n2) v[c * RB + n2] = cmulc(twiddle<M>(n2 * k1), v[c * RB + n2]);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int n2 = 0; n2 < RB; ++n2) buf[lo * P + (g * CB + c) * RB + n2] = v[c * RB + n2];
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < RA; ++k1) v[k1] = buf[lo * P + k1 * RB + g];
    dft<RA, -1>(v);
    // v[n1] = row ky=lo, x = RB*n1 + g; transpose back to buf[ky][x]
    __syncthreads();
#pragma unroll
    for (int n1 = 0; n1 < RA; ++n1) buf[lo * P + RB * n1 + g] = v[n1];
    __syncthreads();
    // ---- inverse, columns; lo = x again
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int k2 = 0; k2 < RB; ++k2) v[c * RB + k2] = buf[((g * CB + c) + RA * k2) * P + lo];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      dft<RB, -1>(&v[c * RB]);
      const int k1 = g * CB + c;
#pragma unroll
      for (int n2 = 1; n2 < RB; ++n2) v[c * RB + n2] = cmulc(twiddle<M>(n2 * k1), v[c * RB + n2]);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int n2 = 0; n2 < RB; ++n2) buf[((g * CB + c) * RB + n2) * P + lo] = v[c * RB + n2];
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < RA; ++k1) v[k1] = buf[(k1 * RB + g) * P + lo];
    dft<RA, -1>(v);

    // ---- R_k = v / M^2; gradient g0 = conj(Q) (Q z_k - R_k)  (eq. 2.2)
    constexpr float inv_m2 = 1.0f / (float)(M * M);
#pragma unroll
    for (int n1 = 0; n1 < RA; ++n1) {
      const int y = RB * n1 + g;
      const float2 qq = a.q[y * M + lo];
      const float2 zz = zp[(size_t)y * a.n_cols];
      const float2 r = cscale(v[n1], inv_m2);
      v[n1] = cmulc(qq, csub(cmul(qq, zz), r));
    }

    if constexpr (MODE == MODE_OBJECTIVE) {
      double gs = 0.0;
#pragma unroll
      for (int n1 = 0; n1 < RA; ++n1) gs += (double)v[n1].x * v[n1].x + (double)v[n1].y * v[n1].y;
      double tot = block_sum<TPB>(gs, red);
      if (tid == 0) a.gnorm_k[k] = sqrt(tot);
      return;
    } else {
      // ---- MAGPS V-cycle, gradient form (FP64 on the coarse grids)
      float2* outp = a.stage + (size_t)blockIdx.x * M * M + lo;
      const int L = a.levels;
      if (L <= 1) {
#pragma unroll
        for (int n1 = 0; n1 < RA; ++n1) outp[(RB * n1 + g) * M] = make_float2(-v[n1].x, -v[n1].y);
        return;
      }
      __syncthreads();
#pragma unroll
      for (int n1 = 0; n1 < RA; ++n1) buf[(RB * n1 + g) * P + lo] = v[n1];
      __syncthreads();
      constexpr int M1 = M / 2;
      constexpr int E1 = (M1 * M1) / TPB;  // level-1 elements per thread (RA / 4)
      double2 gh1[E1];
#pragma unroll
      for (int i = 0; i < E1; ++i) {
        const int e = tid + i * TPB;
        const int Y = e / M1, X = e % M1;
        const float2 p0 = buf[(2 * Y) * P + 2 * X], p1 = buf[(2 * Y) * P + 2 * X + 1];
        const float2 p2 = buf[(2 * Y + 1) * P + 2 * X], p3 = buf[(2 * Y + 1) * P + 2 * X + 1];
        gh1[i].x = 0.25 * (((double)p0.x + p1.x) + ((double)p2.x + p3.x));
        gh1[i].y = 0.25 * (((double)p0.y + p1.y) + ((double)p2.y + p3.y));
      }
      __syncthreads();
      double2* C = smem_d2;  // coarse grids, level l at offset sum_{j<l} (M>>j)^2 (j >= 1)
      // level 1 constants
      const double* V1 = a.lvl;
      const double* rho1 = a.lvl + M1 * M1;
      const double* r1 = a.lvl + 2 * M1 * M1;
      if (L == 2) {
#pragma unroll
        for (int i = 0; i < E1; ++i) {
          const int e = tid + i * TPB;
          const double rr = r1[e];
          C[e] = make_double2(-rr * gh1[i].x, -rr * gh1[i].y);
        }
      } else {
#pragma unroll
        for (int i = 0; i < E1; ++i) C[tid + i * TPB] = gh1[i];
        // restriction down: g^_l = I(V_{l-1} g^_{l-1}); coarsest: e = -r g^
        int off_prev = 0, lv_prev = 0;
        int Mp = M1;
        for (int l = 2; l < L; ++l) {
          __syncthreads();
          const int Ml = Mp >> 1;
          const int off_cur = off_prev + Mp * Mp;
          const int lv_cur = lv_prev + 3 * Mp * Mp;
          const double* Vp = a.lvl + lv_prev;
          const double* rl = a.lvl + lv_cur + 2 * Ml * Ml;
          for (int e = tid; e < Ml * Ml; e += TPB) {
            const int Y = e / Ml, X = e % Ml;
            const int c0 = off_prev + (2 * Y) * Mp + 2 * X, c1 = c0 + Mp;
            const int i0 = (2 * Y) * Mp + 2 * X, i1 = i0 + Mp;
            double2 s;
            s.x = 0.25 * ((Vp[i0] * C[c0].x + Vp[i0 + 1] * C[c0 + 1].x) + (Vp[i1] * C[c1].x + Vp[i1 + 1] * C[c1 + 1].x));
            s.y = 0.25 * ((Vp[i0] * C[c0].y + Vp[i0 + 1] * C[c0 + 1].y) + (Vp[i1] * C[c1].y + Vp[i1 + 1] * C[c1 + 1].y));
            if (l == L - 1) {
              const double rr = rl[e];
              s.x = -rr * s.x;
              s.y = -rr * s.y;
            }
            C[off_cur + e] = s;
          }
          off_prev = off_cur;
          lv_prev = lv_cur;
          Mp = Ml;
        }
        // prolongation up: e_l = rho_l P(e_{l+1}) - r_l g^_l, levels L-2 .. 1
        // (off_prev, lv_prev, Mp) describe level L-1 here
        for (int l = L - 2; l >= 1; --l) {
          __syncthreads();
          const int Ml = Mp << 1;
          const int off_cur = off_prev - Ml * Ml;
          const int lv_cur = lv_prev - 3 * Ml * Ml;
          const double* rhol = a.lvl + lv_cur + Ml * Ml;
          const double* rl = a.lvl + lv_cur + 2 * Ml * Ml;
          for (int e = tid; e < Ml * Ml; e += TPB) {
            const int Y = e / Ml, X = e % Ml;
            const double2 ec = C[off_prev + (Y >> 1) * Mp + (X >> 1)];
            const double2 gh = C[off_cur + e];
            const double rh = rhol[e], rr = rl[e];
            C[off_cur + e] = make_double2(rh * ec.x - rr * gh.x, rh * ec.y - rr * gh.y);
          }
          off_prev = off_cur;
          lv_prev = lv_cur;
          Mp = Ml;
        }
      }
      __syncthreads();
      // level 0: c_k = u0 P(e_1) - g0
#pragma unroll
      for (int n1 = 0; n1 < RA; ++n1) {
        const int y = RB * n1 + g;
        const double2 e1 = C[(y >> 1) * M1 + (lo >> 1)];
        const double uu = (double)a.u0f[y * M + lo];
        outp[y * M] = make_float2((float)(uu * e1.x - (double)v[n1].x), (float)(uu * e1.y - (double)v[n1].y));
      }
    }
  }
}

template <int M>
static hipError_t launch_step_m(int mode, const StepArgs& a, hipStream_t s) {
  constexpr int TPB = M * Plan<M>::RB;
  const size_t lds = (size_t)M * (M + 1) * sizeof(float2);
  if (a.count <= 0) return hipSuccess;
  switch (mode) {
    case MODE_STEP:
      hipFuncSetAttribute((const void*)step_kernel<M, MODE_STEP>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL((step_kernel<M, MODE_STEP>), dim3(a.count), dim3(TPB), lds, s, a);
      break;
    case MODE_OBJECTIVE:
      hipFuncSetAttribute((const void*)step_kernel<M, MODE_OBJECTIVE>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL((step_kernel<M, MODE_OBJECTIVE>), dim3(a.count), dim3(TPB), lds, s, a);
      break;
    case MODE_FORWARD:
      hipFuncSetAttribute((const void*)step_kernel<M, MODE_FORWARD>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL((step_kernel<M, MODE_FORWARD>), dim3(a.count), dim3(TPB), lds, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int step_threads(int m) {
  switch (m) {
    case 8: return 8 * Plan<8>::RB;
    case 16: return 16 * Plan<16>::RB;
    case 32: return 32 * Plan<32>::RB;
    case 64: return 64 * Plan<64>::RB;
    case 128: return 128 * Plan<128>::RB;
    default: return 0;
  }
}

size_t step_lds_bytes(int m) { return (size_t)m * (m + 1) * sizeof(float2); }

hipError_t launch_step(int m, int mode, const StepArgs& a, hipStream_t s) {
  switch (m) {
    case 8: return launch_step_m<8>(mode, a, s);
    case 16: return launch_step_m<16>(mode, a, s);
    case 32: return launch_step_m<32>(mode, a, s);
    case 64: return launch_step_m<64>(mode, a, s);
    case 128: return launch_step_m<128>(mode, a, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Deterministic segmented accumulation + apply.  One workgroup per 64 x 16
// tile; lane = column, wave w owns rows w, w+4, w+8, w+12.  Positions
// overlapping the tile are visited in ascending index; those in minibatch t
// contribute their staged c_k and w0 (FP64 sums).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(ACC_THREADS) void accumulate_kernel(AccumArgs a) {
  constexpr int RPT = ACC_TILE_H / (ACC_THREADS / 64);
  const int tile = blockIdx.x;
  const int tx = tile % a.tiles_x, ty = tile / a.tiles_x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int X = tx * ACC_TILE_W + lane;
  const int Y0 = ty * ACC_TILE_H + wave;
  const int m = a.m;
  double nr[RPT], ni[RPT], dd[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) nr[i] = ni[i] = dd[i] = 0.0;
  const int beg = a.tile_ptr[tile], end = a.tile_ptr[tile + 1];
  const int lo_idx = a.batch_index * a.batch;
  for (int idx = beg; idx < end; ++idx) {
    const int k = a.tile_pos[idx];
    const int slot = a.inv[k] - lo_idx;
    if (slot < 0 || slot >= a.batch) continue;
    const int2 off = a.offs[k];
    const int xx = X - off.y;
    if ((unsigned)xx >= (unsigned)m) continue;
    const float2* sp = a.stage + (size_t)slot * m * m + xx;
    const double* wp = a.w0 + xx;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int yy = Y0 + 4 * i - off.x;
      if ((unsigned)yy < (unsigned)m) {
        const float2 c = sp[(size_t)yy * m];
        nr[i] += (double)c.x;
        ni[i] += (double)c.y;
        dd[i] += wp[yy * m];
      }
    }
  }
  if (X < a.n_cols) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int Y = Y0 + 4 * i;
      if (Y < a.n_rows && dd[i] > 0.0) {
        float2* zp = a.z + (size_t)Y * a.n_cols + X;
        const float2 zo = *zp;
        *zp = make_float2((float)((double)zo.x + nr[i] / dd[i]), (float)((double)zo.y + ni[i] / dd[i]));
      }
    }
  }
}

hipError_t launch_accumulate(const AccumArgs& a, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(accumulate_kernel, dim3(n_tiles), dim3(ACC_THREADS), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Probe hierarchy in FP64 (eq. 4.4, Alg 3 coarse-level preparation).  One
// workgroup.  Level 0: u0 (u^rPIE unless given), w0 = u0 + |Q|^2, FP32 copies.
// Level l >= 1 from level l-1 on 2x2 bins: Q_l = I Q, S = I |Q|^2,
// u^ = I u, w^ = I w, V = |Q_l|^2 / S (0 where S = 0), u_l = V u^;
// rho = u^ / w^, r = 1 / w^ where V > 0 and w^ > 0, else rho = 1, r = 0.
// Output per level: V [Ml^2], rho [Ml^2], r [Ml^2].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void level_constants_kernel(int m, int levels, double alpha, int u_given,
                                                               const double2* q64, double* u0, double* w0,
                                                               float* u0f, float2* qf, double* lvl,
                                                               double2* scr_q, double* scr_u) {
  __shared__ double red[1024];
  const int tid = threadIdx.x;
  const int n0 = m * m;
  double mx = 0.0;
  for (int e = tid; e < n0; e += blockDim.x) {
    const double2 q = q64[e];
    mx = fmax(mx, q.x * q.x + q.y * q.y);
  }
  red[tid] = mx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
    __syncthreads();
  }
  const double amax = red[0];
  for (int e = tid; e < n0; e += blockDim.x) {
    const double2 q = q64[e];
    const double a2 = q.x * q.x + q.y * q.y;
    const double uu = u_given ? u0[e] : alpha * (amax - a2);
    u0[e] = uu;
    w0[e] = uu + a2;
    u0f[e] = (float)uu;
    qf[e] = make_float2((float)q.x, (float)q.y);
  }
  __syncthreads();
  const double2* Qp = q64;
  const double* Up = u0;
  double2* Qn = scr_q;
  double* Un = scr_u;
  int Mp = m;
  int lv = 0;
  for (int l = 1; l < levels; ++l) {
    const int Ml = Mp >> 1;
    double* V = lvl + lv;
    double* rho = V + Ml * Ml;
    double* r = V + 2 * Ml * Ml;
    for (int e = tid; e < Ml * Ml; e += blockDim.x) {
      const int Y = e / Ml, X = e % Ml;
      double2 qs = make_double2(0.0, 0.0);
      double S = 0.0, U = 0.0;
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const int i = (2 * Y + dy) * Mp + 2 * X + dx;
          const double2 q = Qp[i];
          qs.x += q.x;
          qs.y += q.y;
          S += q.x * q.x + q.y * q.y;
          U += Up[i];
        }
      qs.x *= 0.25;
      qs.y *= 0.25;
      S *= 0.25;
      U *= 0.25;
      const double W = U + S;
      const double qa2 = qs.x * qs.x + qs.y * qs.y;
      const double Vv = S > 0.0 ? qa2 / S : 0.0;
      const bool ok = (Vv > 0.0) && (W > 0.0);
      V[e] = Vv;
      rho[e] = ok ? U / W : 1.0;
      r[e] = ok ? 1.0 / W : 0.0;
      Qn[e] = qs;
      Un[e] = Vv * U;
    }
    __syncthreads();
    // next level reads Qn/Un; ping-pong between the two halves of the scratch
    Qp = Qn;
    Up = Un;
    Qn = (Qn == scr_q) ? scr_q + (m / 2) * (m / 2) : scr_q;
    Un = (Un == scr_u) ? scr_u + (m / 2) * (m / 2) : scr_u;
    lv += 3 * Ml * Ml;
    Mp = Ml;
  }
}

hipError_t launch_level_constants(int m, int levels, double alpha, int u_given, const double2* q64,
                                  double* u0, double* w0, float* u0f, float2* qf, double* lvl,
                                  double2* scr_q, double* scr_u, hipStream_t s) {
  hipLaunchKernelGGL(level_constants_kernel, dim3(1), dim3(1024), 0, s, m, levels, alpha, u_given, q64, u0,
                     w0, u0f, qf, lvl, scr_q, scr_u);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// sqrt(d) into kernel order: thread tid = ky + M*g of position k reads
// kx = g*CB + c + RA*k2 for j = c*RB + k2 and writes dst[k][tid*RA + j].
// Flags negative or non-finite input.
// ---------------------------------------------------------------------------
template <int M>
__global__ void permute_sqrt_kernel(int n_pos, const float* src, int is_sqrt, float* dst, int* bad) {
  constexpr int RB = Plan<M>::RB, RA = Plan<M>::RA, CB = RA / RB;
  const int k = blockIdx.x;
  const int tid = threadIdx.x;
  const int ky = tid & (M - 1), g = tid / M;
  const float* sp = src + (size_t)k * M * M + (size_t)ky * M;
  float* dp = dst + (size_t)k * M * M + (size_t)tid * RA;
  int badl = 0;
#pragma unroll
  for (int c = 0; c < CB; ++c)
#pragma unroll
    for (int k2 = 0; k2 < RB; ++k2) {
      float x = sp[g * CB + c + RA * k2];
      if (!(x >= 0.0f) || !isfinite(x)) badl = 1;
      dp[c * RB + k2] = is_sqrt ? x : sqrtf(x);
    }
  if (badl) atomicOr(bad, 1);
}

hipError_t launch_permute_sqrt(int m, int n_pos, const float* src, int is_sqrt, float* dst, int* bad,
                               hipStream_t s) {
  switch (m) {
#define MG_CASE(MM)                                                                                  \
  case MM:                                                                                           \
    hipLaunchKernelGGL(permute_sqrt_kernel<MM>, dim3(n_pos), dim3(MM * Plan<MM>::RB), 0, s, n_pos, src, \
                       is_sqrt, dst, bad);                                                           \
    break;
    MG_CASE(8) MG_CASE(16) MG_CASE(32) MG_CASE(64) MG_CASE(128)
#undef MG_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed-order FP64 sum of n values (one workgroup): thread t sums t, t+256, ...
// in order, then a fixed tree.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void reduce_sum_kernel(const double* x, int n, double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t launch_reduce_sum(const double* x, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(256), 0, s, x, n, out);
  return hipGetLastError();
}

__global__ void convert_c64_c128_kernel(const float2* src, double2* dst, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = make_double2(src[i].x, src[i].y);
}
__global__ void convert_c128_c64_kernel(const double2* src, float2* dst, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = make_float2((float)src[i].x, (float)src[i].y);
}
__global__ void check_finite_c64_kernel(const float2* src, size_t n, int* bad) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && (!isfinite(src[i].x) || !isfinite(src[i].y))) atomicOr(bad, 1);
}

hipError_t launch_convert_c64_c128(const float2* src, double2* dst, size_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(convert_c64_c128_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}
hipError_t launch_convert_c128_c64(const double2* src, float2* dst, size_t n, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(convert_c128_c64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}
hipError_t launch_check_finite_c64(const float2* src, size_t n, int* bad, hipStream_t s) {
  if (!n) return hipSuccess;
  hipLaunchKernelGGL(check_finite_c64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, n, bad);
  return hipGetLastError();
}

}  // namespace mg
