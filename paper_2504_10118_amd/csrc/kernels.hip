// gfx950 kernels of the MAGPIE hot path (arXiv 2504.10118).
//
// step_kernel<M, RB, MODE>  one workgroup per scan position: gather z_k, exit wave
//                       Q * z_k, LDS-resident 2-D FFT, modulus replacement
//                       (Definition 2.1) kept as the difference F(Q z_k) - F(R_k),
//                       inverse FFT of it, gradient
//                       g0 = conj(Q)(Q z_k - R_k) (eq. 2.2), MAGPS V-cycle in
//                       gradient form (Alg 3 / eq. 4.6), write c_k = w0 * dz_k.
// accumulate_kernel     one workgroup per 32 x TH object tile: fixed-order sum
//                       of the overlapping c_k and of w0 (FP64), z += N / D.
// level_constants_kernel FP64 probe hierarchy (eq. 4.4) and per-level
//                       coefficients of the gradient-form V-cycle.
//
// 2-D FFT layout.  M = RA * RB.  A workgroup has M * RB threads; thread
// tid = g + RB * col.  Each 1-D pass along an axis is two register stages:
// stage A, a radix-RA DFT over the RA elements RB apart that a thread holds,
// then the twiddle W_M^(n2 k1); stage B, CB = RA / RB radix-RB DFTs after
// the RB threads of a transform have exchanged data through LDS.  Columns
// are transformed first (col = x), rows second (col = ky), with one LDS
// transpose between.  The forward output lands with thread (ky, g) holding
// kx = g*CB + c + RA*k2, the order sqrt(d) is stored in, so the irreducible
// sqrt(d) stream is read as contiguous per-thread vectors.  The inverse
// retraces the forward steps and returns the data to the gather layout
// (thread (x, g) holds rows y = RB*n1 + g).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

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

// FFT plan: RB threads per 1-D transform, RA = M / RB points per thread
// (RA >= RB), PAD = row padding of the LDS transpose tile in float2.
//
// LDS banks: 64 banks of 4 bytes; the lanes of a 64-bit access are served 32 at
// a time (a float2 slot s sits in bank pair s mod 32), those of a 128-bit access
// 16 at a time.  With 8 threads per transform a wave holds 8 columns (column
// passes) or 8 rows (row passes) of the tile, and lane (cl, g) = (lane / 8,
// lane % 8).  For M >= 64 an odd pitch M + 5 makes the column-slice exchanges
// and the gathers conflict-free and leaves the transposes one extra cycle per
// access, and the row-slice exchange stores a wave's values point-major,
// slot n2 * PX + cl * RA + k1 from the first row of its slice (PX = M + 1 at
// M = 64, M + 2 at M = 128, where the stores pair into 128-bit writes): both its
// stores (k1 fixed) and its loads (n2 fixed) then spread over all bank pairs.
// Smaller plans keep pitch M + 2 and the row-major exchange (cl * P + k1 * RB + n2).
template <int M, int RB_>
struct Plan {
  static constexpr int RB = RB_, RA = M / RB_;
  static constexpr bool WIDE = (M >= 64 && RB_ == 8);
  static constexpr int PAD = WIDE ? 5 : 2;
  static constexpr int PX = M == 64 ? M + 1 : M + 2;
  static_assert(RA >= RB && RA % RB == 0, "stage B needs RA a multiple of RB");
  static_assert(!WIDE || 7 * PX + M <= 8 * (M + PAD), "row-slice exchange exceeds the wave's rows");
};

template <int M>
__device__ __forceinline__ float2 twiddle(int j) {
  return g_twiddle[(j & (M - 1)) * (128 / M)];
}

constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x / 2); }

// M <= 64 keeps Q and u0 in registers from the gather to the V-cycle and
// reads the probe table once, as (Re Q, Im Q, u0, 0) float4s.  Larger M
// re-reads Q and u0 where they are used, so its table holds Q as float2s
// followed by u0 as floats (both in thread order): a re-read fetches only the
// bytes it needs.
constexpr bool keeps_table(int M) { return M <= 64; }

// w[j] = W_M^(b j) for 0 < j < R: the power-of-two exponents are read from
// the table, every other one is the product of its highest power of two and
// the remainder.
template <int M, int R>
__device__ __forceinline__ void powers(int b, float2 (&w)[R]) {
#pragma unroll
  for (int j = 1; j < R; j <<= 1) w[j] = twiddle<M>(b * j);
#pragma unroll
  for (int j = 3; j < R; ++j) {
    if ((j & (j - 1)) == 0) continue;
    const int hb = 1 << ilog2c(j);   // highest power of two <= j
    w[j] = cmul(w[hb], w[j - hb]);
  }
}

constexpr int cst_count_max(int M, int LW) { return cst_count(M, LW + 1); }

// Deepest in-wave V-cycle (number of coarse levels, at most LW) whose constants
// fit in LDS beside the M x P tile.
constexpr int LDS_MAX_BYTES = 160 * 1024;
constexpr int inwave_levels(int M, int P, int LW) {
  int lw = LW;
  while (lw > 0) {
    const long c = (long)cst_count(M, lw + 1) * 8, t = (long)M * P * 8;
    if (t + c <= LDS_MAX_BYTES) break;
    --lw;
  }
  return lw;
}

// Coarse levels of the in-wave V-cycle of a plan (0: the V-cycle runs through LDS).
// At M >= 128 every thread holds 16 points of a column, so the in-wave form would
// repeat each level's FP64 work in all 4^l threads of a bin and stage up to 136 KB
// of constants per workgroup; the LDS form computes each coarse bin once
// (1024 x 1024 object, 128 x 128 probe, 256 positions per launch: 38.7 -> 35.7 us).
constexpr int VCYCLE_LDS_MIN_M = 128;
template <int M, int RB>
constexpr int inwave_depth() {
  constexpr int TPB = M * RB, P = M + Plan<M, RB>::PAD;
  constexpr int LW = ilog2c((TPB < 64 ? TPB : 64) / RB);
  return M >= VCYCLE_LDS_MIN_M ? 0 : inwave_levels(M, P, LW);
}

// Argument blocks read from memory through the constant address space: the
// loads are scalar and the compiler may re-read a field instead of keeping it
// live, so a descriptor costs no vector registers.
template <typename T>
using const_ptr = const __attribute__((address_space(4))) T*;

__device__ __forceinline__ StepArgs load_step_args(const StepArgs* p) {
  const const_ptr<StepArgs> d = (const_ptr<StepArgs>)p;
  StepArgs a;
  a.z = d->z;
  a.n_rows = d->n_rows;
  a.n_cols = d->n_cols;
  a.q = d->q;
  a.sqrtd = d->sqrtd;
  a.offs = d->offs;
  a.pos = d->pos;
  a.posx = nullptr;    // multi-context runs keep workgroup = slot
  a.perm = d->perm;
  a.epoch = d->epoch;
  a.epoch_stride = d->epoch_stride;
  a.count = d->count;
  a.stage = d->stage;
  a.u0f = d->u0f;
  a.qtab = d->qtab;
  a.qspec = d->qspec;
  a.lvl = d->lvl;
  a.lvl_a_off = d->lvl_a_off;
  a.levels = d->levels;
  a.phi_part = d->phi_part;
  a.gn_part = d->gn_part;
  a.d_out = d->d_out;
  a.probe_num = d->probe_num;
  a.probe_den = d->probe_den;
  a.probe_max = d->probe_max;
  a.phase = nullptr;   // multi-context runs do not recycle phases
  a.stage_wt = 0;      // ... and stage through L2 (their launches are large)
  return a;
}

__device__ __forceinline__ AccumArgs load_accum_args(const AccumArgs* p) {
  const const_ptr<AccumArgs> d = (const_ptr<AccumArgs>)p;
  AccumArgs a;
  a.z = d->z;
  a.n_rows = d->n_rows;
  a.n_cols = d->n_cols;
  a.m = d->m;
  a.tiles_x = d->tiles_x;
  a.box_x0 = d->box_x0;
  a.box_y0 = d->box_y0;
  a.box_nx = d->box_nx;
  a.n_tiles = d->n_tiles;
  a.tile_ptr = d->tile_ptr;
  a.tile_ent = d->tile_ent;
  a.pos = d->pos;
  a.count = d->count;
  a.inv = d->inv;
  a.epoch = d->epoch;
  a.epoch_stride = d->epoch_stride;
  a.batch_index = d->batch_index;
  a.batch = d->batch;
  a.stage = d->stage;
  a.offs = d->offs;
  a.w0f = d->w0f;
  return a;
}

// Orders this wave's LDS accesses around the call (LDS executes one wave's
// operations in issue order; the fences keep the compiler from moving them).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over the lanes of one wave (LANES active lanes, a power of two), fixed
// order: butterflies over lane distances LANES / 2, ..., 1 (VALU: which form of
// the cross-lane exchange, see xor_lane).
template <int LANES, int VALU>
__device__ __forceinline__ double wave_sum(double v) {
  if constexpr (LANES >= 64) v += xor_lane<32, VALU>(v);
  if constexpr (LANES >= 32) v += xor_lane<16, VALU>(v);
  if constexpr (LANES >= 16) v += xor_lane<8, VALU>(v);
  if constexpr (LANES >= 8) v += xor_lane<4, VALU>(v);
  if constexpr (LANES >= 4) v += xor_lane<2, VALU>(v);
  if constexpr (LANES >= 2) v += xor_lane<1, VALU>(v);
  return v;
}

template <int LANES, int VALU>
__device__ __forceinline__ float wave_max(float v) {
  auto x = [](float a, auto mask) {
    return __int_as_float(xor_lane<decltype(mask)::value, VALU>(__float_as_int(a)));
  };
  if constexpr (LANES >= 64) v = fmaxf(v, x(v, std::integral_constant<int, 32>{}));
  if constexpr (LANES >= 32) v = fmaxf(v, x(v, std::integral_constant<int, 16>{}));
  if constexpr (LANES >= 16) v = fmaxf(v, x(v, std::integral_constant<int, 8>{}));
  if constexpr (LANES >= 8) v = fmaxf(v, x(v, std::integral_constant<int, 4>{}));
  if constexpr (LANES >= 4) v = fmaxf(v, x(v, std::integral_constant<int, 2>{}));
  if constexpr (LANES >= 2) v = fmaxf(v, x(v, std::integral_constant<int, 1>{}));
  return v;
}

// Modulus replacement of one spectrum value t = F(Q z_k) with measured
// amplitude s (Definition 2.1), kept as the difference t - s e with e = t / |t|
// (= F(Q z_k) - F(R_k)); returns false where t counts as zero (the caller applies
// its theta(0) rule) only where t is exactly zero.  (|t| - s)^2 is added to
// phis, in the accumulator's type PA: FP64 for the objective, FP32 for the per-step
// terms of a step (each thread sums at most 16 of them before the FP64 sum over the
// workgroup, about 1e-6 relative, below the FP32 transform's own error).  The
// hardware reciprocal square root does not take single-precision
// denormals, and |t|^2 underflows for |t| < 2^-75, so where |t|^2 < 2^-100 the
// value is first scaled by 2^100 (exactly): every nonzero t then has a normal
// squared magnitude in [2^-98, 2^100).
template <typename PA>
__device__ __forceinline__ bool modulus_diff(float2 t, float s, float2& out, float2& e, PA& phis) {
  const float a2 = t.x * t.x + t.y * t.y;
  if (a2 >= 0x1p-100f) {
    const float ra = __builtin_amdgcn_rsqf(a2);
    const PA dlt = (PA)(a2 * ra) - (PA)s;
    phis += dlt * dlt;
    e = make_float2(t.x * ra, t.y * ra);
    const float f = fmaf(-s, ra, 1.0f);
    out = make_float2(t.x * f, t.y * f);
    return true;
  }
  const float tx = t.x * 0x1p100f, ty = t.y * 0x1p100f;
  const float b2 = tx * tx + ty * ty;
  if (!(b2 > 0.0f)) return false;
  const float rb = __builtin_amdgcn_rsqf(b2);
  const PA dlt = (PA)(b2 * rb) * (PA)0x1p-100 - (PA)s;
  phis += dlt * dlt;
  e = make_float2(tx * rb, ty * rb);
  out = make_float2(fmaf(-s, e.x, t.x), fmaf(-s, e.y, t.y));
  return true;
}

// MAGPS V-cycle through LDS for hierarchies whose coarse bins span several
// waves.  On entry g0 is in T[y][x] (pitch P) and in v (thread (x, g) holds
// rows RB*n1 + g), and u0v holds u0 at the same pixels.  Coarse grids (FP64)
// overwrite the start of the LDS tile: level 1 with rows padded to M / 2 + 1 (the
// final prolongation reads 4 rows of it per 16 lanes, in 4 different banks), then
// levels 2.. unpadded.  Each level's constants (V, rho, r: they do not depend on
// the data) are loaded before the barrier that precedes the level, so their
// latency overlaps the wait.
template <int M, int TPB, int P, int RB, int RA>
__device__ void magps_lds(const StepArgs& a, const float2* T, double2* C, const float2* v, const float* u0v,
                          int col, int g, float2* stage_k, const int tid) {
  const int L = a.levels;
  constexpr int M1 = M / 2, S1 = M1 + 1;
  constexpr int E1 = (M1 * M1 + TPB - 1) / TPB;               // level-1 bins per thread
  constexpr int E2 = ((M / 4) * (M / 4) + TPB - 1) / TPB;     // bins per thread on levels >= 2
  // level l's grid: offset and row pitch in C
  auto off_of = [&](int l) {
    int o = 0;
    for (int j = 1; j < l; ++j) o += (j == 1) ? M1 * S1 : (M >> j) * (M >> j);
    return o;
  };
  auto pitch_of = [&](int l) { return l == 1 ? S1 : (M >> l); };
  // Three or four grids: one lane per level-2 bin does the whole hierarchy for its
  // bin.  Wave w holds the 8 x 8 block (w % BW, w / BW) of level-2 bins, its lane bits
  // (x0, y0, x1, y1, x2, y2) give the bin inside the block, so a level-3 bin is the
  // four lanes that differ in bits 0 and 1 (its restriction two cross-lane sums, its
  // prolongation free).  The lane reads the 4 x 4 gradient pixels of its bin from the
  // tile, forms g^_1 of its four level-1 children and g^_2, goes down to the coarsest
  // level and back, and writes e_1 of its children: one barrier (every lane has read
  // its pixels before C, which overlays the tile, is written) instead of one per level
  // and direction.  Sums in the same pairing and order as the path through LDS below.
  // (Levels 4 and 5 fit the same block, but carrying them in registers spilled at the
  // 128-register cap: deeper hierarchies take the LDS path.)
  constexpr int M2 = M / 4, BW = M2 / 8;
  constexpr bool WAVE_OK = (M2 >= 8) && (BW * BW * 64 <= TPB);
  if (WAVE_OK && (L == 3 || L == 4)) {
    const int wv = tid >> 6, lane = tid & 63;
    const bool act = wv < BW * BW;
    const int X2 = (act ? (wv % BW) * 8 : 0) + ((lane & 1) | ((lane >> 1) & 2) | ((lane >> 2) & 4));
    const int Y2 = (act ? (wv / BW) * 8 : 0) + (((lane >> 1) & 1) | ((lane >> 2) & 2) | ((lane >> 3) & 4));
    auto lv_of = [&](int l) {   // offset of level l's (V, rho, r) block in a.lvl
      int o = 0;
      for (int j = 1; j < l; ++j) o += 3 * (M >> j) * (M >> j);
      return o;
    };
    auto at = [&](int l, int which) {   // V (0), rho (1) or r (2) of level l >= 2 at this lane's bin
      const int Ml = M >> l, sh = l - 2;
      return a.lvl[lv_of(l) + which * Ml * Ml + (Y2 >> sh) * Ml + (X2 >> sh)];
    };
    // level-1 constants of the four children (i0, i0 + 1, i1, i1 + 1) and the coarse ones
    const int i0 = (2 * Y2) * M1 + 2 * X2, i1 = i0 + M1;
    const int ci[4] = {i0, i0 + 1, i1, i1 + 1};
    double v1[4], rh1[4], rr1[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v1[q] = a.lvl[ci[q]];
      rh1[q] = a.lvl[M1 * M1 + ci[q]];
      rr1[q] = a.lvl[2 * M1 * M1 + ci[q]];
    }
    const double v2 = (L == 4) ? at(2, 0) : 0.0;
    const double rh2 = (L == 4) ? at(2, 1) : 0.0, rr2 = (L == 4) ? at(2, 2) : 0.0;
    const double rc = at(L - 1, 2);
    double2 e1[4];
    if (act) {
      // g^_1 of the children from their 2 x 2 gradient pixels
      double2 ch[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int Y = 2 * Y2 + (q >> 1), X = 2 * X2 + (q & 1);
        const float2 p0 = T[(2 * Y) * P + 2 * X], p1 = T[(2 * Y) * P + 2 * X + 1];
        const float2 p2 = T[(2 * Y + 1) * P + 2 * X], p3 = T[(2 * Y + 1) * P + 2 * X + 1];
        ch[q].x = 0.25 * (((double)p0.x + p1.x) + ((double)p2.x + p3.x));
        ch[q].y = 0.25 * (((double)p0.y + p1.y) + ((double)p2.y + p3.y));
      }
      double2 g2;
      g2.x = 0.25 * ((v1[0] * ch[0].x + v1[1] * ch[1].x) + (v1[2] * ch[2].x + v1[3] * ch[3].x));
      g2.y = 0.25 * ((v1[0] * ch[0].y + v1[1] * ch[1].y) + (v1[2] * ch[2].y + v1[3] * ch[3].y));
      double2 e;
      if (L == 4) {
        // g^_3 = I(V_2 g^_2) over the four lanes of the level-3 bin; coarsest e_3 = -r_3 g^_3;
        // e_2 = rho_2 P(e_3) - r_2 g^_2
        const double2 t = make_double2(v2 * g2.x, v2 * g2.y);
        const double2 o = xor_lane<1>(t);
        const double2 sx = make_double2(t.x + o.x, t.y + o.y);
        const double2 w = xor_lane<2>(sx);
        const double2 g3 = make_double2(0.25 * (sx.x + w.x), 0.25 * (sx.y + w.y));
        const double2 e3 = make_double2(-rc * g3.x, -rc * g3.y);
        e = make_double2(rh2 * e3.x - rr2 * g2.x, rh2 * e3.y - rr2 * g2.y);
      } else {
        e = make_double2(-rc * g2.x, -rc * g2.y);   // level 2 is the coarsest
      }
      // e_1 = rho_1 P(e_2) - r_1 g^_1 for the four children
#pragma unroll
      for (int q = 0; q < 4; ++q)
        e1[q] = make_double2(rh1[q] * e.x - rr1[q] * ch[q].x, rh1[q] * e.y - rr1[q] * ch[q].y);
    }
    __syncthreads();   // every lane has read its pixels: C may overwrite the tile
    if (act) {
      const int c0 = (2 * Y2) * S1 + 2 * X2, c1 = c0 + S1;
      C[c0] = e1[0];
      C[c0 + 1] = e1[1];
      C[c1] = e1[2];
      C[c1 + 1] = e1[3];
    }
  } else {
    // two grids: level 1 is the coarsest, e_1 = -r_1 g^_1 (r_1 follows V_1, rho_1)
    const double* r1 = a.lvl + 2 * M1 * M1;
    double r1v[E1];
    double2 gh1[E1];
  #pragma unroll
    for (int i = 0; i < E1; ++i) {
      const int e = tid + i * TPB;
      r1v[i] = (L == 2 && e < M1 * M1) ? r1[e] : 0.0;
      gh1[i] = make_double2(0.0, 0.0);
      if (e < M1 * M1) {
        const int Y = e / M1, X = e % M1;
        const float2 p0 = T[(2 * Y) * P + 2 * X], p1 = T[(2 * Y) * P + 2 * X + 1];
        const float2 p2 = T[(2 * Y + 1) * P + 2 * X], p3 = T[(2 * Y + 1) * P + 2 * X + 1];
        gh1[i].x = 0.25 * (((double)p0.x + p1.x) + ((double)p2.x + p3.x));
        gh1[i].y = 0.25 * (((double)p0.y + p1.y) + ((double)p2.y + p3.y));
      }
    }
    __syncthreads();
  #pragma unroll
    for (int i = 0; i < E1; ++i) {
      const int e = tid + i * TPB;
      if (e < M1 * M1) {
        double2 w = gh1[i];
        if (L == 2) w = make_double2(-r1v[i] * w.x, -r1v[i] * w.y);
        C[(e / M1) * S1 + e % M1] = w;
      }
    }
    // restriction down: g^_l = I(V_{l-1} g^_{l-1}); coarsest: e = -r g^
    int lv_prev = 0, Mp = M1;
    for (int l = 2; l < L; ++l) {
      const int Ml = Mp >> 1;
      const int off_prev = off_of(l - 1), sp = pitch_of(l - 1), off_cur = off_of(l);
      const int lv_cur = lv_prev + 3 * Mp * Mp;
      const double* Vp = a.lvl + lv_prev;
      const double* rl = a.lvl + lv_cur + 2 * Ml * Ml;
      double vq[E2][4], rq[E2];
  #pragma unroll
      for (int i = 0; i < E2; ++i) {
        const int e = tid + i * TPB;
        rq[i] = 0.0;
        vq[i][0] = vq[i][1] = vq[i][2] = vq[i][3] = 0.0;
        if (e < Ml * Ml) {
          const int Y = e / Ml, X = e % Ml;
          const int i0 = (2 * Y) * Mp + 2 * X, i1 = i0 + Mp;
          vq[i][0] = Vp[i0];
          vq[i][1] = Vp[i0 + 1];
          vq[i][2] = Vp[i1];
          vq[i][3] = Vp[i1 + 1];
          if (l == L - 1) rq[i] = rl[e];
        }
      }
      __syncthreads();
  #pragma unroll
      for (int i = 0; i < E2; ++i) {
        const int e = tid + i * TPB;
        if (e < Ml * Ml) {
          const int Y = e / Ml, X = e % Ml;
          const int c0 = off_prev + (2 * Y) * sp + 2 * X, c1 = c0 + sp;
          double2 s;
          s.x = 0.25 * ((vq[i][0] * C[c0].x + vq[i][1] * C[c0 + 1].x) + (vq[i][2] * C[c1].x + vq[i][3] * C[c1 + 1].x));
          s.y = 0.25 * ((vq[i][0] * C[c0].y + vq[i][1] * C[c0 + 1].y) + (vq[i][2] * C[c1].y + vq[i][3] * C[c1 + 1].y));
          if (l == L - 1) {
            s.x = -rq[i] * s.x;
            s.y = -rq[i] * s.y;
          }
          C[off_cur + e] = s;
        }
      }
      lv_prev = lv_cur;
      Mp = Ml;
    }
    // prolongation up: e_l = rho_l P(e_{l+1}) - r_l g^_l for l = L-2 .. 1
    for (int l = L - 2; l >= 1; --l) {
      const int Ml = Mp << 1;
      const int off_prev = off_of(l + 1), sp = pitch_of(l + 1), off_cur = off_of(l), sc = pitch_of(l);
      const int lv_cur = lv_prev - 3 * Ml * Ml;
      const double* rhol = a.lvl + lv_cur + Ml * Ml;
      const double* rl = a.lvl + lv_cur + 2 * Ml * Ml;
      double rh[E1], rr[E1];
  #pragma unroll
      for (int i = 0; i < E1; ++i) {
        const int e = tid + i * TPB;
        const bool in = e < Ml * Ml;
        rh[i] = in ? rhol[e] : 0.0;
        rr[i] = in ? rl[e] : 0.0;
      }
      __syncthreads();
  #pragma unroll
      for (int i = 0; i < E1; ++i) {
        const int e = tid + i * TPB;
        if (e < Ml * Ml) {
          const int Y = e / Ml, X = e % Ml;
          const double2 ec = C[off_prev + (Y >> 1) * sp + (X >> 1)];
          const double2 gh = C[off_cur + Y * sc + X];
          C[off_cur + Y * sc + X] = make_double2(rh[i] * ec.x - rr[i] * gh.x, rh[i] * ec.y - rr[i] * gh.y);
        }
      }
      lv_prev = lv_cur;
      Mp = Ml;
    }
  }
  __syncthreads();
  // stage_k (this position's staged update) is uniform, so the resource stays scalar
  const rsrc_t outr = make_rsrc(stage_k, (unsigned)(M * M * sizeof(float2)));
#pragma unroll
  for (int n1 = 0; n1 < RA; ++n1) {
    const int y = RB * n1 + g;
    const double2 e1 = C[(y >> 1) * S1 + (col >> 1)];
    const double uu = (double)u0v[n1];
    bstore2_stage(outr, make_float2((float)(uu * e1.x - (double)v[n1].x), (float)(uu * e1.y - (double)v[n1].y)),
                  (y * M + col) * (int)sizeof(float2), 0, a.stage_wt != 0);
  }
}

// Per-position kernel.  Thread tid = g + RB * col (g in [0, RB), col in [0, M)):
// in column passes `col` is the image column x, in row passes it is the
// frequency row ky.  A wave holds CPW = 64 / RB consecutive columns (rows).
// Every LDS access of a wave stays inside its own column slice (column passes)
// or its own row slice (row passes) of the transpose tile T, so the register
// stages exchange data through LDS without workgroup barriers; only the two
// transposes (forward and back) synchronise the workgroup.
// COH: the object is read at device scope (the work-queue launch, where other
// workgroups of the same launch update it).
template <int M, int RBv, int MODE, bool COH = false>
__device__ __forceinline__ void step_body(const StepArgs& a, const int wg) {
  constexpr int RB = Plan<M, RBv>::RB, RA = Plan<M, RBv>::RA;
  constexpr int TPB = M * RB, CB = RA / RB, P = M + Plan<M, RBv>::PAD;
  constexpr int LANES = TPB < 64 ? TPB : 64;
  constexpr int CPW = LANES / RB;
  constexpr int LRB = ilog2c(RB), LW = ilog2c(CPW);
  constexpr int LWI = inwave_depth<M, RBv>();    // coarse levels handled inside the wave
  constexpr int NW = (TPB + 63) / 64;
  // cross-lane exchanges in VALU form while the plan runs few waves per SIMD
  // (up to 512 threads); the 1024-thread plans, whose LDS pipe and VALU are both
  // about half busy, keep distances 4 and 16 in the LDS pipe (measured: all in
  // VALU form +4 us per launch on the 1024 x 1024 object with the 128 x 128 probe, 4 or 16 as well +0.3-0.8 us, 32 alone -0.2 us)
  constexpr int XV = TPB <= 512 ? XOR_ALL_VALU : 32;
  extern __shared__ double2 smem_d2[];
  float2* T = reinterpret_cast<float2*>(smem_d2);

  // In the work-queue launch the body runs in a loop: an opaque copy of the
  // thread index keeps the compiler from hoisting the index arithmetic out of
  // the loop and holding it in registers across both item kinds.
  int tid = threadIdx.x;
  if constexpr (COH) asm volatile("" : "+v"(tid));
  const int g = tid & (RB - 1);
  const int col = tid / RB;
  const int cl = col & (CPW - 1);
  const int c0w = col - cl;
  const int wave = tid >> 6;
  const size_t eoff = a.epoch ? (size_t)(*a.epoch) * a.epoch_stride : 0;
  int k, slot = wg;   // slot: where this position's staged update (and probe partials) go
  int2 off;
  if (a.posx) {
    const int4 pr = a.posx[eoff + wg];
    k = pr.x;
    off = make_int2(pr.y, pr.z);
    slot = pr.w;
  } else if (a.pos) {
    const int4 pr = a.pos[eoff + wg];
    k = pr.x;
    off = make_int2(pr.y, pr.z);
  } else {
    k = a.perm ? a.perm[eoff + wg] : (int)wg;
    off = a.offs[k];
  }
  if constexpr (COH) {
    // loaded inside the queue's loop these are vector loads (earlier items' stores
    // may alias them); the values are uniform, and the buffer resources built
    // from them must be scalar
    k = __builtin_amdgcn_readfirstlane(k);
    slot = __builtin_amdgcn_readfirstlane(slot);
    off = make_int2(__builtin_amdgcn_readfirstlane(off.x), __builtin_amdgcn_readfirstlane(off.y));
  }

  // exchange index inside the wave's slice: (cl, k1, n2) -> [0, 64 * RA)
  auto xi = [&](int k1, int n2) { return (cl * RA + k1) * RB + n2; };
  auto colslice = [&](int i) { return T + (i / CPW) * P + c0w + (i & (CPW - 1)); };
  auto rowslice = [&](int i) { return T + (c0w + i / M) * P + (i & (M - 1)); };
  // row-slice exchange slot of this thread's value (k1, n2)
  auto rx = [&](int k1, int n2) {
    if constexpr (Plan<M, RBv>::WIDE) return T + c0w * P + n2 * Plan<M, RBv>::PX + cl * RA + k1;
    else return rowslice(xi(k1, n2));
  };

  // ---- gather z_k, exit wave Q * z_k: thread (x = col, g) holds rows y = RB*n1 + g
  float2 v[RA];
  // patch rows y = RB*n1 + g: per-lane byte offset (g, col), per-row scalar offset n1
  const float2* zbase = a.z + (size_t)off.x * a.n_cols + off.y;
  const rsrc_t zr = make_rsrc(zbase, (unsigned)(((size_t)(a.n_rows - off.x) * a.n_cols - off.y) * sizeof(float2)));
  const int zvo = (g * a.n_cols + col) * (int)sizeof(float2);
  const int zso = RB * a.n_cols * (int)sizeof(float2);
  constexpr int ZPOL = COH ? kPolicyDeviceScope : 0;
  constexpr int qso = RB * M * (int)sizeof(float2);
  const float4* qt = a.qtab + tid;   // [n1][tid]: each load reads one contiguous block
  const float2* qt2 = reinterpret_cast<const float2*>(a.qtab) + tid;            // split table: Q
  const float* ut = reinterpret_cast<const float*>(reinterpret_cast<const float2*>(a.qtab) + M * M) + tid;  // u0
  // M <= 64 keeps Q and u0 in registers for the gradient conj(Q)(Q z_k - R_k)
  // and the V-cycle output; M = 128 (1024 threads at the 128-register cap)
  // re-reads its table entries there instead.
  constexpr bool KEEP = keeps_table(M);
  constexpr bool PREQ = (RA <= 8);        // probe table entries in flight with the gather
  // MODE_STEP_PR is the object step with the eq. (3.2) phase store
  constexpr bool STEPM = (MODE == MODE_STEP) || (MODE == MODE_STEP_PR);
  // in-wave V-cycle constants parked in LDS beside the tile (M <= 64; larger M
  // takes the V-cycle through LDS, which reads its constants from memory)
  constexpr bool CST = STEPM && (M <= 64) && (LWI > 0);
  // The twiddle table reads go first (small, needed by the first FFT stage).
  float2 qk[KEEP ? RA : 1];
  float u0k[KEEP ? RA : 1];
  float4 qtv[PREQ ? RA : 1];
  // twiddles: stage A uses W_M^(g k1); the inverse stage B uses W_M^(n2 (g CB + c)).
  // Powers of two of the base come from the table, the other exponents are
  // products of two earlier ones (at most log2 RA roundings deep).
  // At M = 128 (16 points per thread, 128 VGPRs) they are re-formed at each use
  // and sqrt(d) is fetched just before the row pass instead of at the start.
  constexpr bool LAZY = (M >= 128);
  float2 twA[RA];
  auto load_twA = [&]() { powers<M, RA>(g, twA); };
  load_twA();
  float sd[RA];
  auto load_sd = [&]() {
    if constexpr (MODE != MODE_FORWARD) {
      const rsrc_t sr = make_rsrc(a.sqrtd + (size_t)k * M * M, (unsigned)(M * M * sizeof(float)));
#pragma unroll
      for (int i = 0; i < RA / 4; ++i) {
        const float4 t = bload4(sr, tid * RA * (int)sizeof(float), i * 16);
        sd[4 * i] = t.x; sd[4 * i + 1] = t.y; sd[4 * i + 2] = t.z; sd[4 * i + 3] = t.w;
      }
    }
  };
  // In-wave V-cycle constants (A_l, V_l; M <= 64): fetched as 16-byte pairs
  // (the block starts at an even offset and is padded by one double) right
  // after the patch, parked in LDS at the first barrier, so their latency
  // hides behind the forward FFT.
  constexpr int M1c = M / 2;
  constexpr int CST_MAX = CST ? cst_count_max(M, LWI) : 2;
  constexpr int CST_PER = ((CST_MAX + 1) / 2 + TPB - 1) / TPB;   // double2 per thread
  double* const Cst = reinterpret_cast<double*>(T + M * P);
  const int nCst = (CST && a.levels >= 2 && a.levels - 1 <= LWI) ? cst_count(M, a.levels) : 0;
  double2 cst[CST_PER];
  auto load_cst = [&]() {
    if constexpr (CST) {
      const double2* src = reinterpret_cast<const double2*>(a.lvl + a.lvl_a_off);
#pragma unroll
      for (int i = 0; i < CST_PER; ++i) {
        const int e = tid + i * TPB;
        cst[i] = (2 * e < nCst) ? src[e] : make_double2(0.0, 0.0);
      }
    }
  };

  // Gather: the patch is read as whole rows (each wave reads contiguous row
  // segments) into the LDS tile, and after one barrier every thread takes its
  // column values (rows y = RB*n1 + g of column col) from it; the tile is then
  // reused by the FFT.  (Each wave loading its own columns directly, with no
  // barrier, measured slower at 256 and at 1600 positions per launch.)
  // Row gather: load j of thread tid reads row tid / M + j * TPB / M, column
  // tid % M: one per-lane offset, and a uniform per-load row step.
  constexpr int GR = TPB / M;   // rows per load of the workgroup
  auto row_gather = [&]() {
    const int gvo = ((tid / M) * a.n_cols + (tid & (M - 1))) * (int)sizeof(float2);
    const int gso = GR * a.n_cols * (int)sizeof(float2);
    float2* const dst = T + (tid / M) * P + (tid & (M - 1));
#pragma unroll
    for (int j = 0; j < RA; ++j) dst[j * GR * P] = bload2p<ZPOL>(zr, gvo, j * gso);
  };
  row_gather();
  // The probe table (needed with the patch), the constants (parked in LDS
  // before the first transpose) and sqrt(d) (needed at the modulus) are issued
  // after the patch, in the order they are needed: loads return in issue
  // order, so issued first they had held up the patch the barrier below waits
  // for (512 x 512 object, 64 x 64 probe: epoch -2 % for sqrt(d) and the constants, -1.3 % for the
  // table, -0.6 % for the constants ahead of sqrt(d)).
  if constexpr (PREQ) {
#pragma unroll
    for (int n1 = 0; n1 < RA; ++n1) qtv[n1] = qt[n1 * TPB];
  }
  load_cst();
  if constexpr (!LAZY) load_sd();
  __syncthreads();
  // reference value of the window: its centre pixel (see the spectrum term after
  // the forward transform, which reads it back from s_zc past the next barrier
  // rather than holding it in registers through the column pass)
  __shared__ float2 s_zc;
  const float2 zc = T[(M / 2) * P + M / 2];
  if (tid == 0) s_zc = zc;
#pragma unroll
  for (int n1 = 0; n1 < RA; ++n1) {
    float2 qv;
    float uv = 0.0f;
    if constexpr (KEEP) {
      const float4 t = PREQ ? qtv[n1] : qt[n1 * TPB];
      qv = make_float2(t.x, t.y);
      uv = t.z;
    } else {
      qv = qt2[n1 * TPB];
    }
    const float2 zz = T[(RB * n1 + g) * P + col];
    v[n1] = cmul(qv, make_float2(zz.x - zc.x, zz.y - zc.y));   // Q (z_k - z_c); z_c F(Q) is added after the transform
    if constexpr (KEEP) {
      qk[n1] = qv;
      u0k[n1] = uv;
    }
  }
  wave_sync();   // the column pass below reuses this wave's own column slice of the tile

  // ---- forward, columns: stage A (radix RA over n1), twiddle, exchange, stage B
  dft<RA, 1>(v);
#pragma unroll
  for (int k1 = 1; k1 < RA; ++k1) v[k1] = cmul(v[k1], twA[k1]);
#pragma unroll
  for (int k1 = 0; k1 < RA; ++k1) *colslice(xi(k1, g)) = v[k1];
  wave_sync();
#pragma unroll
  for (int c = 0; c < CB; ++c)
#pragma unroll
    for (int n2 = 0; n2 < RB; ++n2) v[c * RB + n2] = *colslice(xi(g * CB + c, n2));
#pragma unroll
  for (int c = 0; c < CB; ++c) dft<RB, 1>(&v[c * RB]);
  wave_sync();
  // v[c*RB + k2] = column spectrum at ky = g*CB + c + RA*k2; transpose into T[ky][x]
#pragma unroll
  for (int c = 0; c < CB; ++c)
#pragma unroll
    for (int k2 = 0; k2 < RB; ++k2) T[((g * CB + c) + RA * k2) * P + col] = v[c * RB + k2];
  if constexpr (CST) {
#pragma unroll
    for (int i = 0; i < CST_PER; ++i)
      if (2 * (tid + i * TPB) < nCst) reinterpret_cast<double2*>(Cst)[tid + i * TPB] = cst[i];
  }
  __syncthreads();

  // ---- forward, rows (col = ky now): stage A over x = RB*n1 + g
  if constexpr (LAZY) load_sd();
#pragma unroll
  for (int n1 = 0; n1 < RA; ++n1) v[n1] = T[col * P + RB * n1 + g];
  if constexpr (LAZY) load_twA();
  dft<RA, 1>(v);
#pragma unroll
  for (int k1 = 1; k1 < RA; ++k1) v[k1] = cmul(v[k1], twA[k1]);
  wave_sync();
#pragma unroll
  for (int k1 = 0; k1 < RA; ++k1) *rx(k1, g) = v[k1];
  wave_sync();
#pragma unroll
  for (int c = 0; c < CB; ++c)
#pragma unroll
    for (int n2 = 0; n2 < RB; ++n2) v[c * RB + n2] = *rx(g * CB + c, n2);
  // v[c*RB + k2] = F(Q (z_k - z_c))[ky = col][kx = g*CB + c + RA*k2]; adding z_c F(Q) gives
  // Psi = F(Q z_k) (exact for any scalar z_c).  A window that is nearly constant
  // (the flat start above all) has exit waves close to a multiple of Q, whose far
  // field spans more than FP32 resolves in one transform (dark pixels would take
  // their phase from rounding); with the probe's spectrum computed once in FP64 the
  // transform only carries the departure from the window's centre value, whose
  // size is that of the variation of z_k (never that of 1 - z_k: tiny objects
  // stay exact).  The spectrum is added group by group after each RB-point DFT,
  // so that only RB of its values are live at a time.
  // Buffer loads: one per-lane offset and a constant per-load offset (a plain
  // pointer per load costs an address pair each and spilled at 128 x 128).
  const float2 zcs = s_zc;
  const rsrc_t qsr = make_rsrc(a.qspec, (unsigned)(M * M * sizeof(float2)));
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    dft<RB, 1>(&v[c * RB]);
    if constexpr (LAZY) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k2 = 0; k2 < RB; ++k2) {
      const float2 r = cmul(zcs, bload2(qsr, tid * (int)sizeof(float2), (c * RB + k2) * TPB * (int)sizeof(float2)));
      v[c * RB + k2] = make_float2(v[c * RB + k2].x + r.x, v[c * RB + k2].y + r.y);
    }
  }

  if constexpr (MODE == MODE_FORWARD) {
    float* dp = a.d_out + (size_t)k * M * M + (size_t)col * M;
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int k2 = 0; k2 < RB; ++k2) {
        const float2 t = v[c * RB + k2];
        dp[g * CB + c + RA * k2] = t.x * t.x + t.y * t.y;
      }
    return;
  } else {
    // ---- modulus replacement (Definition 2.1, theta(0) = 0); Phi_k partial (summed
    // in FP64 for the objective; for a step's own terms per thread in FP32, then FP64).
    // The spectrum is replaced by the difference F(Q z_k) - F(R_k) = F(Q z_k)
    // (1 - sqrt(d) / |F(Q z_k)|) (-sqrt(d) theta where the spectrum vanishes), so
    // the inverse transform yields Q z_k - R_k itself: the gradient needs
    // neither the exit wave kept nor the patch read again.
    using PA = std::conditional_t<MODE == MODE_OBJECTIVE, double, float>;
    PA phis = 0;
    if constexpr (MODE == MODE_STEP_PR) {
      // eq. (3.2): every phase factor is kept for the position's next visit and
      // read back where the spectrum vanishes exactly (theta = 0 before the
      // first visit: the store starts as 1).  Natural order: row ky = col,
      // column kx = g*CB + c + RA*k2 for j = c*RB + k2.
      float2* const ph = a.phase + (size_t)k * M * M + (size_t)col * M;
#pragma unroll
      for (int j = 0; j < RA; ++j) {
        const int kx = g * CB + j / RB + RA * (j % RB);
        const float s = sd[j];
        float2 e, dv;
        if (modulus_diff(v[j], s, dv, e, phis)) {
          ph[kx] = e;
          v[j] = dv;
        } else {
          phis += (PA)s * (PA)s;
          e = ph[kx];
          v[j] = make_float2(-s * e.x, -s * e.y);
        }
      }
    } else {
#pragma unroll
    for (int j = 0; j < RA; ++j) {
      const float s = sd[j];
      float2 e, dv;
      if (modulus_diff(v[j], s, dv, e, phis)) {
        v[j] = dv;
      } else {
        phis += (PA)s * (PA)s;
        v[j] = make_float2(-s, 0.0f);
      }
    }
    }
    if (a.phi_part) {
      const double tot = wave_sum<LANES, XV>((double)phis);
      if ((tid & 63) == 0) a.phi_part[(size_t)k * MAX_WAVES + wave] = tot * (0.5 / ((double)M * (double)M));
    }

    // ---- inverse, rows: stage B^-1, conj twiddle, exchange, stage A^-1
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      dft<RB, -1>(&v[c * RB]);
      float2 twB[RB];
      if constexpr (CB == 1) {
#pragma unroll
        for (int n2 = 1; n2 < RB; ++n2) twB[n2] = twA[n2];
      } else {
        powers<M, RB>(g * CB + c, twB);
      }
#pragma unroll
      for (int n2 = 1; n2 < RB; ++n2) v[c * RB + n2] = cmulc(twB[n2], v[c * RB + n2]);
    }
    wave_sync();
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int n2 = 0; n2 < RB; ++n2) *rx(g * CB + c, n2) = v[c * RB + n2];
    wave_sync();
#pragma unroll
    for (int k1 = 0; k1 < RA; ++k1) v[k1] = *rx(k1, g);
    dft<RA, -1>(v);
    wave_sync();
    // v[n1] = row ky = col at x = RB*n1 + g; transpose back into T[ky][x] (own rows)
#pragma unroll
    for (int n1 = 0; n1 < RA; ++n1) T[col * P + RB * n1 + g] = v[n1];
    __syncthreads();

    // ---- inverse, columns (col = x): stage B^-1 over k2, conj twiddle, exchange, stage A^-1
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int k2 = 0; k2 < RB; ++k2) v[c * RB + k2] = T[((g * CB + c) + RA * k2) * P + col];
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      dft<RB, -1>(&v[c * RB]);
      float2 twB[RB];
      if constexpr (CB == 1) {
#pragma unroll
        for (int n2 = 1; n2 < RB; ++n2) twB[n2] = twA[n2];
      } else {
        powers<M, RB>(g * CB + c, twB);
      }
#pragma unroll
      for (int n2 = 1; n2 < RB; ++n2) v[c * RB + n2] = cmulc(twB[n2], v[c * RB + n2]);
    }
    wave_sync();
#pragma unroll
    for (int c = 0; c < CB; ++c)
#pragma unroll
      for (int n2 = 0; n2 < RB; ++n2) *colslice(xi(g * CB + c, n2)) = v[c * RB + n2];
    wave_sync();
#pragma unroll
    for (int k1 = 0; k1 < RA; ++k1) v[k1] = *colslice(xi(k1, g));
    dft<RA, -1>(v);

    // ---- gradient g0 = conj(Q) (Q z_k - R_k) (eq. 2.2): v / M^2 is Q z_k - R_k
    constexpr float inv_m2 = 1.0f / (float)(M * M);
    float pmx = 0.0f;
#pragma unroll
    for (int n1 = 0; n1 < RA; ++n1) {
      float2 qq;
      if constexpr (KEEP) qq = qk[n1];
      else qq = qt2[n1 * TPB];
      const float2 dk = cscale(v[n1], inv_m2);
      if constexpr (STEPM) {
        if (a.probe_num) {
          // probe step partials: conj(z_k)(R_k - Q z_k) and |z_k|^2 (the patch
          // is read again for them, at the column stride)
          const float2 zz = bload2p<ZPOL>(zr, zvo, n1 * zso);
          const float2 pn = cmulc(zz, make_float2(-dk.x, -dk.y));
          const float pd = zz.x * zz.x + zz.y * zz.y;
          const size_t e = (size_t)slot * M * M + (size_t)(RB * n1 + g) * M + col;
          a.probe_num[e] = pn;
          a.probe_den[e] = pd;
          pmx = fmaxf(pmx, pd);
        }
      }
      v[n1] = cmulc(qq, dk);
    }
    if constexpr (STEPM) {
      if (a.probe_num) {
        const float wm = wave_max<LANES, XV>(pmx);
        if ((tid & 63) == 0) a.probe_max[(size_t)slot * MAX_WAVES + wave] = wm;
      }
    }

    if constexpr (MODE == MODE_OBJECTIVE) {
      double gs = 0.0;
#pragma unroll
      for (int n1 = 0; n1 < RA; ++n1) gs += (double)v[n1].x * v[n1].x + (double)v[n1].y * v[n1].y;
      const double tot = wave_sum<LANES, XV>(gs);
      if ((tid & 63) == 0) a.gn_part[(size_t)k * MAX_WAVES + wave] = tot;
      return;
    } else {
      const rsrc_t outr = make_rsrc(a.stage + (size_t)slot * M * M, (unsigned)(M * M * sizeof(float2)));
      const int ovo = (g * M + col) * (int)sizeof(float2);
      const int L = a.levels;
      if (L <= 1) {
#pragma unroll
        for (int n1 = 0; n1 < RA; ++n1)
          bstore2_stage(outr, make_float2(-v[n1].x, -v[n1].y), ovo, n1 * qso, a.stage_wt != 0);
        return;
      }
      if (L - 1 <= LWI) {
        // ---- MAGPS V-cycle inside the wave (gradient form, FP64).  Level-l
        // values are held replicated by every thread of their 2^l x 2^l bin,
        // so restriction is two cross-lane (or in-thread) pair sums and
        // prolongation is free.  The upward pass is folded into per-level
        // coefficients: e_1 = sum_l A_l g^_l with A_l = -r_l prod_{j<l} rho_j.
        // Chunks of NC register rows: while every restriction pairs rows across
        // lanes (LW <= log2 RB) the rows n1 are independent.
        // in-thread row pairs (levels above log2 RB) stay inside aligned chunks of NC
        constexpr int NCB = (M >= 128) ? 2 : 4;
        constexpr int NCP = (LW > LRB) ? (1 << (LW - LRB)) : 1;
        constexpr int NC0 = NCP > NCB ? NCP : NCB;
        constexpr int NC = NC0 < RA ? NC0 : RA;
#pragma unroll
        for (int n0 = 0; n0 < RA; n0 += NC) {
          double2 cur[NC], e1[NC];
#pragma unroll
          for (int i = 0; i < NC; ++i) {
            cur[i] = make_double2(v[n0 + i].x, v[n0 + i].y);
            e1[i] = make_double2(0.0, 0.0);
          }
#pragma unroll
          for (int l = 1; l <= LWI; ++l) {
            if (l < L) {
              const int Ml = M >> l;
              double2 s[NC];
              if (l == 1) {
                // the partner row's FP32 values, widened after the exchange (half the
                // cross-lane moves of exchanging the FP64 values; the same sums)
#pragma unroll
                for (int i = 0; i < NC; ++i) {
                  const float2 f = v[n0 + i];
                  const float ox = __int_as_float(xor_lane<1, XV>(__float_as_int(f.x)));
                  const float oy = __int_as_float(xor_lane<1, XV>(__float_as_int(f.y)));
                  s[i] = make_double2((double)f.x + (double)ox, (double)f.y + (double)oy);
                }
              } else if (l - 1 < LRB) {
#pragma unroll
                for (int i = 0; i < NC; ++i) {
                  const double2 o = xor_lane_rt<XV>(cur[i], 1 << (l - 1));
                  s[i] = make_double2(cur[i].x + o.x, cur[i].y + o.y);
                }
              } else {
                const int b = (l - 1 >= LRB) ? (1 << (l - 1 - LRB)) : 0;
#pragma unroll
                for (int i = 0; i < NC; ++i) {
                  const double2 o = cur[(i ^ b) & (NC - 1)];
                  s[i] = make_double2(cur[i].x + o.x, cur[i].y + o.y);
                }
              }
              // A_l and V_l from the block parked in LDS (rows padded by CST_PAD), both
              // stored times 1/4: gh is the bin's sum, 4 g^_l, and the products with the
              // scaled constants are the same numbers as those of the mean (scaling by a
              // power of two is exact)
              const double* A = (const double*)Cst + (size_t)(l - 1) * M1c * (M1c + CST_PAD);
              const double* V = (const double*)Cst + cst_v_off(M, L, l);
              const bool more = (l + 1 < L);
#pragma unroll
              for (int i = 0; i < NC; ++i) {
                const double2 o = xor_lane_rt<XV>(s[i], RB << (l - 1));
                const double2 gh = make_double2(s[i].x + o.x, s[i].y + o.y);
                const int y = RB * (n0 + i) + g;
                const double aa = A[(y >> 1) * (M1c + CST_PAD) + (col >> 1)];
                e1[i] = make_double2(e1[i].x + aa * gh.x, e1[i].y + aa * gh.y);
                if (more) {
                  const double vv = V[(y >> l) * (Ml + CST_PAD) + (col >> l)];
                  cur[i] = make_double2(vv * gh.x, vv * gh.y);
                }
              }
            }
          }
          // level 0: c_k = u0 P(e_1) - g0
#pragma unroll
          for (int i = 0; i < NC; ++i) {
            const int y = RB * (n0 + i) + g;
            double uu;
            if constexpr (KEEP) uu = (double)u0k[n0 + i];
            else uu = (double)ut[(n0 + i) * TPB];
            bstore2_stage(outr,
                          make_float2((float)(uu * e1[i].x - (double)v[n0 + i].x),
                                      (float)(uu * e1[i].y - (double)v[n0 + i].y)),
                          ovo, (n0 + i) * qso, a.stage_wt != 0);
          }
        }
        return;
      }
      // ---- deep hierarchies (coarse bins wider than a wave): V-cycle through LDS.
      // u0 of this thread's pixels: from registers, or (M = 128) from the
      // thread-ordered table, loaded here so that the V-cycle hides the latency.
      float u0v[RA];
#pragma unroll
      for (int n1 = 0; n1 < RA; ++n1) {
        if constexpr (KEEP) u0v[n1] = u0k[n1];
        else u0v[n1] = ut[n1 * TPB];
      }
      __syncthreads();
#pragma unroll
      for (int n1 = 0; n1 < RA; ++n1) T[(RB * n1 + g) * P + col] = v[n1];
      __syncthreads();
      magps_lds<M, TPB, P, RB, RA>(a, T, smem_d2, v, u0v, col, g, a.stage + (size_t)slot * M * M, tid);
    }
  }
}


template <int M, int RBv, int MODE>
__global__ __launch_bounds__(M * RBv) void step_kernel(StepArgs a) {
  step_body<M, RBv, MODE>(a, (int)blockIdx.x);
}

// Many reconstructions in one launch: workgroup b belongs to the context j with
// prefix[j] <= b < prefix[j + 1] (prefix: running totals of the contexts' work
// items for this round, so contexts with none take no workgroups), and does its
// item b - prefix[j].  The search is uniform across the workgroup.
__device__ __forceinline__ int owner_of(const int* __restrict__ prefix, int n_ctx, int b) {
  int lo = 0, hi = n_ctx;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <int M, int RBv>
__global__ __launch_bounds__(M * RBv) void step_multi_kernel(const StepArgs* __restrict__ descs,
                                                             const int* __restrict__ prefix, int n_ctx) {
  const int b = (int)blockIdx.x;
  const int j = owner_of(prefix, n_ctx, b);
  const StepArgs a = load_step_args(descs + j);
  step_body<M, RBv, MODE_STEP>(a, b - prefix[j]);
}

template <int M, int RB>
constexpr size_t lds_bytes_c() {
  constexpr int P = M + Plan<M, RB>::PAD;
  constexpr int LW = inwave_depth<M, RB>();
  size_t b = (size_t)M * P * sizeof(float2);
  const size_t c = (size_t)((cst_count_max(M, LW) + 1) & ~1) * sizeof(double);
  b += c;                       // in-wave constants parked beside the tile (none where LW = 0)
  return b;
}
template <int M, int RB>
static size_t lds_bytes_m() {
  static_assert(lds_bytes_c<M, RB>() <= (size_t)LDS_MAX_BYTES, "step kernel LDS exceeds the CU's LDS");
  return lds_bytes_c<M, RB>();
}

template <int M, int RB, int MODE>
static hipError_t launch_step_mode(const StepArgs& a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  constexpr int TPB = M * RB;
  const size_t lds = lds_bytes_m<M, RB>();
  const hipError_t e =
      hipFuncSetAttribute((const void*)step_kernel<M, RB, MODE>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (ev0)
    hipExtLaunchKernelGGL((step_kernel<M, RB, MODE>), dim3(a.count), dim3(TPB), lds, s, ev0, ev1, 0, a);
  else
    hipLaunchKernelGGL((step_kernel<M, RB, MODE>), dim3(a.count), dim3(TPB), lds, s, a);
  return hipGetLastError();
}

template <int M, int RB>
static hipError_t launch_step_p(int mode, const StepArgs& a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (a.count <= 0) return hipSuccess;
  switch (mode) {
    case MODE_STEP:
      return a.phase ? launch_step_mode<M, RB, MODE_STEP_PR>(a, s, ev0, ev1)
                     : launch_step_mode<M, RB, MODE_STEP>(a, s, ev0, ev1);
    case MODE_OBJECTIVE: return launch_step_mode<M, RB, MODE_OBJECTIVE>(a, s, ev0, ev1);
    case MODE_FORWARD: return launch_step_mode<M, RB, MODE_FORWARD>(a, s, ev0, ev1);
    default: return hipErrorInvalidValue;
  }
}

// The compiled plans: (M, RB).  The first plan listed for an M is its default.
#define MG_FOR_EACH_PLAN(X) X(8, 2) X(16, 4) X(16, 2) X(32, 4) X(32, 2) X(64, 8) X(64, 4) X(128, 8) X(128, 4)

bool plan_valid(int m, int rb) {
#define MG_PV(MM, RR) if (m == MM && rb == RR) return true;
  MG_FOR_EACH_PLAN(MG_PV)
#undef MG_PV
  return false;
}

int default_plan(int m) {
  switch (m) {
    case 8: return 2;
    case 16: return 4;
    case 32: return 4;
    case 64: return 8;
    case 128: return 8;
    default: return 0;
  }
}

int plans_for(int m, int* rbs, int cap) {
  int n = 0;
#define MG_PL(MM, RR) if (m == MM && n < cap) rbs[n++] = RR;
  MG_FOR_EACH_PLAN(MG_PL)
#undef MG_PL
  return n;
}

hipError_t launch_step(int m, int rb, int mode, const StepArgs& a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
#define MG_LS(MM, RR) if (m == MM && rb == RR) return launch_step_p<MM, RR>(mode, a, s, ev0, ev1);
  MG_FOR_EACH_PLAN(MG_LS)
#undef MG_LS
  return hipErrorInvalidValue;
}

int step_threads(int m, int rb) { return plan_valid(m, rb) ? m * rb : 0; }
int step_waves(int m, int rb) { return (step_threads(m, rb) + 63) / 64; }

size_t step_lds_bytes(int m, int rb) {
#define MG_LB(MM, RR) if (m == MM && rb == RR) return lds_bytes_m<MM, RR>();
  MG_FOR_EACH_PLAN(MG_LB)
#undef MG_LB
  return 0;
}

// ---------------------------------------------------------------------------
// Deterministic segmented accumulation + apply.  One workgroup per 32 x TH
// tile; a wave covers two rows (lanes 0-31 and 32-63 = columns), wave w owns
// rows 2w, 2w+1, 2w+8, 2w+9, ... .  32-column tiles are overlapped by fewer
// positions than 64-column ones (a window reaches a tile from a 32 + m - 1
// column range instead of 64 + m - 1), so each pixel loops over fewer members
// that do not cover it (512 x 512 object, 64 x 64 probe: epoch -3 % against 64 x 4 tiles).  The positions
// overlapping the tile (ascending index, with their offsets) are screened 256
// at a time in parallel: those in minibatch t are compacted, order preserved,
// into LDS, then every thread sums their staged c_k and w0 over its pixels in
// that order (FP64 sums of the staged FP32 c_k and an FP32 copy of w0).  Loads are predicated
// rather than branched so that several positions' loads are in flight.
// ---------------------------------------------------------------------------
// COH: the staged updates and the object are read, and the object written, at
// device scope (the work-queue launch, where workgroups on other XCDs produce
// and consume them within the launch).
template <int TH, bool COH = false>
__device__ __forceinline__ void accumulate_body(const AccumArgs& a, const int b) {
  constexpr int NT = acc_threads(TH);
  constexpr int NW = NT / 64;
  constexpr int RPT = TH / (2 * NW);   // rows per thread (1)
  constexpr int U = 4;   // positions whose loads are in flight together
  __shared__ int s_slot[NT];
  __shared__ int2 s_off[NT];
  __shared__ int s_wcnt[NW];
  const int tx = a.box_x0 + b % a.box_nx, ty = a.box_y0 + b / a.box_nx;
  const int tile = ty * a.tiles_x + tx;
  int tid = threadIdx.x;
  if constexpr (COH) asm volatile("" : "+v"(tid));   // as in step_body
  const int lane = tid & 63, wave = tid >> 6;
  const int X = tx * ACC_TILE_W + (lane & 31);
  const int Y0 = ty * TH + 2 * wave + (lane >> 5);
  const int m = a.m;
  const size_t mm = (size_t)m * m;
  double nr[RPT], ni[RPT], dd[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) nr[i] = ni[i] = dd[i] = 0.0;
  // the tile's current object values, fetched first: their latency overlaps
  // the screening and the staged loads
  float2 zo[RPT];
  [[maybe_unused]] rsrc_t zrs, srs;
  if constexpr (COH) {
    zrs = make_rsrc(a.z, (unsigned)((size_t)a.n_rows * a.n_cols * sizeof(float2)));
    srs = make_rsrc(a.stage, (unsigned)((size_t)a.batch * m * m * sizeof(float2)));
  }
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int Y = Y0 + 2 * NW * i;
    if constexpr (COH)
      zo[i] = (X < a.n_cols && Y < a.n_rows)
                  ? bload2p<kPolicyDeviceScope>(zrs, (int)((unsigned)(Y * a.n_cols + X) * (unsigned)sizeof(float2)), 0)
                  : make_float2(0.0f, 0.0f);
    else
      zo[i] = (X < a.n_cols && Y < a.n_rows) ? a.z[(size_t)Y * a.n_cols + X] : make_float2(0.0f, 0.0f);
  }
  // candidates: the minibatch's own records (slot = processing index; a window
  // overlaps the tile where it reaches both its column and its row range), or the
  // static list of positions overlapping the tile, kept where the inverse
  // permutation puts them in this minibatch (slot order = ascending position)
  const size_t eoff = a.epoch ? (size_t)(*a.epoch) * a.epoch_stride : 0;
  const bool scan = a.pos != nullptr;
  const int4* recs = scan ? a.pos + eoff : nullptr;
  const int x0 = tx * ACC_TILE_W, y0 = ty * TH;
  const int beg = scan ? 0 : a.tile_ptr[tile], end = scan ? a.count : a.tile_ptr[tile + 1];
  const int lo_idx = a.batch_index * a.batch;
  const int* inv = a.inv + eoff;
  for (int base = beg; base < end; base += NT) {
    const int idx = base + tid;
    int slot = -1;
    int2 off = make_int2(0, 0);
    if (idx < end) {
      if (scan) {
        const int4 pr = recs[idx];
        if (pr.z < x0 + ACC_TILE_W && pr.z + m > x0 && pr.y < y0 + TH && pr.y + m > y0) {
          slot = idx;
          off = make_int2(pr.y, pr.z);
        }
      } else {
        const int4 te = a.tile_ent[idx];
        const int s = inv[te.x] - lo_idx;
        if (s >= 0 && s < a.batch) {
          slot = s;
          off = make_int2(te.y, te.z);
        }
      }
    }
    const bool in = slot >= 0;
    const unsigned long long mask = __ballot(in);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) s_wcnt[wave] = __popcll(mask);
    __syncthreads();
    int wbase = 0, total = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const int c = s_wcnt[w];
      wbase += (w < wave) ? c : 0;
      total += c;
    }
    if (in) {
      s_slot[wbase + before] = slot;
      s_off[wbase + before] = off;
    }
    __syncthreads();
    // sum the compacted entries in order, U positions' loads at a time
    for (int j = 0; j < total; j += U) {
      float2 cv[U][RPT];
      float wv[U][RPT];
      bool ok[U][RPT];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool have = (j + u) < total;
        const int sl = have ? s_slot[j + u] : 0;
        const int2 o = have ? s_off[j + u] : make_int2(-m, -m);
        const int xx = X - o.y;
        const bool okx = have && (unsigned)xx < (unsigned)m;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const int yy = Y0 + 2 * NW * i - o.x;
          ok[u][i] = okx && ((unsigned)yy < (unsigned)m);
          const int e = ok[u][i] ? (yy * m + xx) : 0;
          if constexpr (COH)
            cv[u][i] = bload2p<kPolicyDeviceScope>(srs, (int)(((unsigned)sl * (unsigned)mm + e) * sizeof(float2)), 0);
          else
            cv[u][i] = a.stage[(size_t)sl * mm + e];
          wv[u][i] = a.w0f[e];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int i = 0; i < RPT; ++i)
          if (ok[u][i]) {
            nr[i] += (double)cv[u][i].x;
            ni[i] += (double)cv[u][i].y;
            dd[i] += (double)wv[u][i];
          }
    }
    __syncthreads();
  }
  if (X < a.n_cols) {
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int Y = Y0 + 2 * NW * i;
      if (Y < a.n_rows && dd[i] > 0.0) {
        const float2 zn =
            make_float2((float)((double)zo[i].x + nr[i] / dd[i]), (float)((double)zo[i].y + ni[i] / dd[i]));
        if constexpr (COH)
          bstore2_device(zrs, zn, (int)((unsigned)(Y * a.n_cols + X) * (unsigned)sizeof(float2)), 0);
        else
          a.z[(size_t)Y * a.n_cols + X] = zn;
      }
    }
  }
}

template <int TH>
__global__ __launch_bounds__(acc_threads(TH)) void accumulate_kernel(AccumArgs a) {
  accumulate_body<TH>(a, (int)blockIdx.x);
}

template <int TH>
__global__ __launch_bounds__(acc_threads(TH)) void accumulate_multi_kernel(const AccumArgs* __restrict__ descs,
                                                                       const int* __restrict__ prefix, int n_ctx) {
  const int b = (int)blockIdx.x;
  const int j = owner_of(prefix, n_ctx, b);
  const AccumArgs a = load_accum_args(descs + j);
  accumulate_body<TH>(a, b - prefix[j]);
}

// ---------------------------------------------------------------------------
// Work-queue launch over many reconstructions' rounds (one launch per FFT plan
// and chunk of rounds, in place of a step and an accumulation launch per
// round).  Each workgroup takes the next item from a counter, waits until the
// items it depends on are done, runs it, and counts it done:
//   step item (member j, round r, position b): waits for the accumulation of
//     every tile of j's earlier rounds (it reads the object they wrote, and
//     writes staging slots they read);
//   tile item (member j, round r, tile b, tile height M RB / 32 so that its
//     pixels take all threads): waits for every step of j's rounds up to r.
// Items are queued round by round, steps before tiles, so every item depends
// only on items taken before it: the earliest unfinished item always has its
// dependencies done and is held by a running workgroup, so the queue drains
// whatever the number of resident workgroups.  Data handed between workgroups
// (object, staged updates) is stored and loaded at device scope, which keeps
// it coherent across the XCDs' L2 caches without cache write-back or
// invalidation; a workgroup counts an item done only after its stores have
// completed.  A wait longer than wait_ticks sets the abort flag, after which
// every workgroup stops taking items (the host reports the failure).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int ld_agent(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int add_agent(int* p, int v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Four waves per SIMD (two 512-thread workgroups per CU) for the 64 x 64 plan
// of 8 threads per transform, as for its step kernel (the loop around both item
// kinds otherwise takes one register more than that allows).
constexpr int queue_min_waves(int m, int rb) { return (m == 64 && rb == 8) ? 4 : 1; }

template <int M, int RBv>
__global__ __launch_bounds__(M * RBv, queue_min_waves(M, RBv)) void queue_kernel(QueueArgs q) {
  constexpr int TH = M * RBv / ACC_TILE_W;
  static_assert(acc_threads(TH) == M * RBv && TH >= 2, "tile items take every thread");
  __shared__ int s_item, s_ok;
  const int tid = threadIdx.x;
  const int nm = q.n_members;
  int* prev = nullptr;   // done counter of the item just finished (uniform)
  // each pass takes a distinct index from head, so a workgroup makes at most
  // total + 1 passes; more would mean the queue is broken: stop it
  for (int pass = 0;; ++pass) {
    if (pass > q.total) {
      if (tid == 0) __hip_atomic_store(q.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    // one region of thread 0 per iteration, between barriers: count the last item
    // done (its stores completed before the barrier that ends it), take the next
    if (tid == 0) {
      if (prev) add_agent(prev, 1);
      s_item = ld_agent(q.abort) ? q.total : add_agent(q.head, 1);
    }
    __syncthreads();
    // uniform across the workgroup: the item's descriptors then load into scalar registers
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= q.total) break;
    const int g = owner_of(q.gpre, q.n_groups, it);
    const int gr = g / nm, j = g - gr * nm;
    const int r = gr >> 1, ph = gr & 1;   // ph 0: step item, 1: tile item
    if (tid == 0) {
      const int* ctr = q.done + (size_t)((ph == 0 ? nm : 0) + j) * QSLOTS * QSLOT_STRIDE;
      auto count = [&]() {
        int c = 0;
#pragma unroll
        for (int sl = 0; sl < QSLOTS; ++sl) c += ld_agent(ctr + sl * QSLOT_STRIDE);
        return c;
      };
      const int need = q.wait[g];
      int ok = 1;
      if (count() < need) {
        const long long t0 = (long long)wall_clock64();
        while (count() < need) {
          if (ld_agent(q.abort) || (long long)wall_clock64() - t0 > q.wait_ticks) {
            __hip_atomic_store(q.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ok = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
      s_ok = ok;
    }
    __syncthreads();
    if (!__builtin_amdgcn_readfirstlane(s_ok)) break;
    const int b = __builtin_amdgcn_readfirstlane(it - q.gpre[g]);
    if (ph == 0) {
      StepArgs a = load_step_args(q.sdesc + (size_t)r * nm + j);
      a.stage_wt = 1;   // staged updates at device scope: tile items on other XCDs read them
      step_body<M, RBv, MODE_STEP, true>(a, b);
    } else {
      const AccumArgs a = load_accum_args(q.adesc + (size_t)r * nm + j);
      accumulate_body<TH, true>(a, b);
    }
    prev = q.done + ((size_t)(ph * nm + j) * QSLOTS + (b & (QSLOTS - 1))) * QSLOT_STRIDE;
    __builtin_amdgcn_s_waitcnt(0);   // this thread's stores have completed
    __syncthreads();
  }
}

template <int TH>
static void launch_accumulate_t(const AccumArgs& a, int n_tiles, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (ev0)
    hipExtLaunchKernelGGL(accumulate_kernel<TH>, dim3(n_tiles), dim3(acc_threads(TH)), 0, s, ev0, ev1, 0, a);
  else
    hipLaunchKernelGGL(accumulate_kernel<TH>, dim3(n_tiles), dim3(acc_threads(TH)), 0, s, a);
}

bool tile_valid(int th) { return th == 8 || th == 16 || th == 32; }

hipError_t launch_step_multi(int m, int rb, const StepArgs* descs, const int* prefix, int n_ctx, int total,
                             hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (n_ctx <= 0 || total <= 0) return hipSuccess;
#define MG_LM(MM, RR)                                                                                   \
  if (m == MM && rb == RR) {                                                                            \
    const size_t lds = lds_bytes_m<MM, RR>();                                                           \
    const hipError_t fe = hipFuncSetAttribute((const void*)step_multi_kernel<MM, RR>,                   \
                                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
    if (fe != hipSuccess) return fe;                                                                    \
    if (ev0)                                                                                            \
      hipExtLaunchKernelGGL((step_multi_kernel<MM, RR>), dim3(total), dim3(MM * RR), lds, s, ev0, ev1, 0, \
                            descs, prefix, n_ctx);                                                      \
    else                                                                                                \
      hipLaunchKernelGGL((step_multi_kernel<MM, RR>), dim3(total), dim3(MM * RR), lds, s, descs, prefix, n_ctx); \
    return hipGetLastError();                                                                           \
  }
  MG_FOR_EACH_PLAN(MG_LM)
#undef MG_LM
  return hipErrorInvalidValue;
}

template <int TH>
static void launch_acc_multi_t(const AccumArgs* descs, const int* prefix, int n_ctx, int total, hipStream_t s,
                               hipEvent_t ev0, hipEvent_t ev1) {
  if (ev0)
    hipExtLaunchKernelGGL(accumulate_multi_kernel<TH>, dim3(total), dim3(acc_threads(TH)), 0, s, ev0, ev1, 0, descs,
                          prefix, n_ctx);
  else
    hipLaunchKernelGGL(accumulate_multi_kernel<TH>, dim3(total), dim3(acc_threads(TH)), 0, s, descs, prefix, n_ctx);
}

hipError_t launch_accumulate_multi(int th, const AccumArgs* descs, const int* prefix, int n_ctx, int total,
                                   hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (n_ctx <= 0 || total <= 0) return hipSuccess;
  switch (th) {
    case 8: launch_acc_multi_t<8>(descs, prefix, n_ctx, total, s, ev0, ev1); break;
    case 16: launch_acc_multi_t<16>(descs, prefix, n_ctx, total, s, ev0, ev1); break;
    case 32: launch_acc_multi_t<32>(descs, prefix, n_ctx, total, s, ev0, ev1); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int qtile_rows(int m, int rb) {
  if (!plan_valid(m, rb)) return 0;
  const int th = m * rb / ACC_TILE_W;
  return th >= 2 ? th : 0;
}

__global__ void clear_i32_kernel(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

hipError_t clear_i32(int* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(clear_i32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

template <int M, int RB>
static hipError_t launch_queue_t(const QueueArgs& q, int n_cu, hipStream_t s) {
  if constexpr (M * RB / ACC_TILE_W < 2) {
    return hipErrorInvalidValue;
  } else {
    const size_t lds = lds_bytes_m<M, RB>();
    hipError_t e = hipFuncSetAttribute((const void*)queue_kernel<M, RB>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, queue_kernel<M, RB>, M * RB, lds);
    if (e != hipSuccess) return e;
    const int grid = std::max(1, std::min(q.total, std::max(1, per_cu) * n_cu));
    hipLaunchKernelGGL((queue_kernel<M, RB>), dim3(grid), dim3(M * RB), lds, s, q);
    return hipGetLastError();
  }
}

hipError_t launch_queue(int m, int rb, const QueueArgs& q, int n_cu, hipStream_t s) {
  if (q.total <= 0) return hipSuccess;
#define MG_LQ(MM, RR) if (m == MM && rb == RR) return launch_queue_t<MM, RR>(q, n_cu, s);
  MG_FOR_EACH_PLAN(MG_LQ)
#undef MG_LQ
  return hipErrorInvalidValue;
}

hipError_t launch_accumulate(const AccumArgs& a, int th, int n_tiles, hipStream_t s, hipEvent_t ev0,
                             hipEvent_t ev1) {
  if (n_tiles <= 0) return hipSuccess;
  switch (th) {
    case 8: launch_accumulate_t<8>(a, n_tiles, s, ev0, ev1); break;
    case 16: launch_accumulate_t<16>(a, n_tiles, s, ev0, ev1); break;
    case 32: launch_accumulate_t<32>(a, n_tiles, s, ev0, ev1); break;
    default: return hipErrorInvalidValue;
  }
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
                                                               float* w0f, float* u0f, float2* qf, double* lvl,
                                                               int a_off, double2* scr_q, double* scr_u) {
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
    w0f[e] = (float)(uu + a2);
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
  // A_l = -r_l prod_{j<l} rho_j along the ancestors of each level-1 bin, so
  // that e_1 = sum_l A_l g^_l (the upward pass of the V-cycle, unrolled).  The
  // in-wave V-cycle's block: A_1..A_{L-1}, then copies of V_1..V_{L-2}, every
  // grid row padded to side + CST_PAD doubles (pads zero), all stored times 1/4
  // (the in-wave V-cycle multiplies them with the sums of 2 x 2 bins, not the means).
  __syncthreads();
  if (levels > 1) {
    const int M1 = m / 2, S1 = M1 + CST_PAD;
    double* A = lvl + a_off;
    for (int e = tid; e < M1 * S1; e += blockDim.x) {
      const int Y1 = e / S1, X1 = e % S1;
      double prod = 1.0;
      int off = 0;
      for (int l = 1; l < levels; ++l) {
        const int Ml = m >> l;
        double val = 0.0;
        if (X1 < M1) {
          const int idx = (Y1 >> (l - 1)) * Ml + (X1 >> (l - 1));
          const double rho = lvl[off + Ml * Ml + idx];
          const double r = lvl[off + 2 * Ml * Ml + idx];
          val = -r * prod;
          prod *= rho;
        }
        A[(size_t)(l - 1) * M1 * S1 + e] = 0.25 * val;
        off += 3 * Ml * Ml;
      }
    }
    double* Vc = lvl + a_off + cst_v_off(m, levels, 1);
    int off = 0;
    for (int l = 1; l <= levels - 2; ++l) {
      const int Ml = m >> l, Sl = Ml + CST_PAD;
      for (int e = tid; e < Ml * Sl; e += blockDim.x) {
        const int Y = e / Sl, X = e % Sl;
        Vc[e] = X < Ml ? 0.25 * lvl[off + Y * Ml + X] : 0.0;
      }
      Vc += Ml * Sl;
      off += 3 * Ml * Ml;
    }
  }
}

// (Re Q, Im Q, u0, 0) per pixel in the thread order of plan (M, RB): entry
// [n1][tid] belongs to thread tid = g + RB*col at pixel (RB*n1 + g, col), so
// each of the step kernel's loads of this table reads one contiguous block.
template <int M, int RB>
__global__ void qtab_kernel(const float2* qf, const float* u0f, float4* qtab) {
  constexpr int TPB = M * RB;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * M) return;
  const int n1 = e / TPB, tid = e - n1 * TPB, g = tid & (RB - 1), col = tid / RB;
  const int i = (RB * n1 + g) * M + col;
  const float2 q = qf[i];
  if constexpr (keeps_table(M)) {
    qtab[e] = make_float4(q.x, q.y, u0f[i], 0.0f);
  } else {
    float2* q2 = reinterpret_cast<float2*>(qtab);
    q2[e] = q;
    reinterpret_cast<float*>(q2 + M * M)[e] = u0f[i];
  }
}

// Probe spectrum F(Q) of the FP32 probe in FP64 (a direct DFT along each axis,
// exact twiddles from sincospi of the reduced exponent), rounded to FP32 once.
// Values within the DFT's own rounding bound, 2 m eps sum |Q| (doubled here), are
// set to exactly zero: a symmetric probe's spectrum vanishes exactly on whole
// lines, where the modulus replacement takes theta(0), and the sums leave there
// only rounding (below 1e-16 sum |Q|, against 1e-8 sum |Q| for the smallest value
// that does not vanish, with the 128 x 128 test probe).
// Rows: one workgroup per row y, thread kx: A[y][kx] = sum_x Q[y][x] W^(kx x);
// the row's sum |Q[y][x]| goes to tmp[m * m + y].x.
__global__ void probe_spectrum_rows_kernel(int m, const float2* __restrict__ qf, double2* __restrict__ tmp) {
  const int y = blockIdx.x, kx = threadIdx.x;
  double re = 0.0, im = 0.0, l1 = 0.0;
  for (int x = 0; x < m; ++x) {
    double sn, cs;
    sincospi(-2.0 * (double)((kx * x) % m) / (double)m, &sn, &cs);
    const float2 q = qf[y * m + x];
    re += (double)q.x * cs - (double)q.y * sn;
    im += (double)q.x * sn + (double)q.y * cs;
    l1 += hypot((double)q.x, (double)q.y);
  }
  tmp[y * m + kx] = make_double2(re, im);
  if (kx == 0) tmp[m * m + y] = make_double2(l1, 0.0);
}
// Columns, written in the plan's spectral thread order: entry e = j * TPB + tid
// holds F[ky][kx] with ky = tid / RB, kx = (tid % RB) * CB + j / RB + RA * (j % RB).
template <int M, int RB>
__global__ void probe_spectrum_cols_kernel(const double2* __restrict__ tmp, float2* __restrict__ qspec) {
  constexpr int TPB = M * RB, RA = M / RB, CB = RA / RB;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * M) return;
  const int j = e / TPB, tid = e - j * TPB;
  const int ky = tid / RB, kx = (tid % RB) * CB + j / RB + RA * (j % RB);
  double re = 0.0, im = 0.0, l1 = 0.0;
  for (int y = 0; y < M; ++y) {
    double sn, cs;
    sincospi(-2.0 * (double)((ky * y) % M) / (double)M, &sn, &cs);
    const double2 t = tmp[y * M + kx];
    re += t.x * cs - t.y * sn;
    im += t.x * sn + t.y * cs;
    l1 += tmp[M * M + y].x;
  }
  const double bound = 4.0 * M * 0x1p-52 * l1;
  qspec[e] = hypot(re, im) <= bound ? make_float2(0.0f, 0.0f) : make_float2((float)re, (float)im);
}

hipError_t launch_level_constants(int m, int levels, double alpha, int u_given, const double2* q64,
                                  double* u0, double* w0, float* w0f, float* u0f, float2* qf, double* lvl,
                                  int lvl_a_off, double2* scr_q, double* scr_u, int rb, float4* qtab,
                                  float2* qspec, double2* spec_tmp, hipStream_t s) {
  hipLaunchKernelGGL(level_constants_kernel, dim3(1), dim3(1024), 0, s, m, levels, alpha, u_given, q64, u0,
                     w0, w0f, u0f, qf, lvl, lvl_a_off, scr_q, scr_u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(probe_spectrum_rows_kernel, dim3(m), dim3(m), 0, s, m, (const float2*)qf, spec_tmp);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
#define MG_QT(MM, RR)                                                                                     \
  if (m == MM && rb == RR) {                                                                              \
    hipLaunchKernelGGL((qtab_kernel<MM, RR>), dim3((MM * MM + 255) / 256), dim3(256), 0, s, qf, u0f, qtab); \
    e = hipGetLastError();                                                                                \
    if (e != hipSuccess) return e;                                                                        \
    hipLaunchKernelGGL((probe_spectrum_cols_kernel<MM, RR>), dim3((MM * MM + 255) / 256), dim3(256), 0, s, \
                       (const double2*)spec_tmp, qspec);                                                  \
    return hipGetLastError();                                                                             \
  }
  MG_FOR_EACH_PLAN(MG_QT)
#undef MG_QT
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// sqrt(d) between natural order [k][ky][kx] and the kernel order of plan
// (M, RB): thread tid = g + RB*ky of position k holds kx = g*CB + c + RA*k2 at
// j = c*RB + k2, i.e. element [k][tid*RA + j].  Natural -> kernel flags
// negative or non-finite input.
// ---------------------------------------------------------------------------
template <int M, int RB, int TO_KERNEL>
__global__ void permute_sqrt_kernel(int n_pos, const float* src, int is_sqrt, float* dst, int* bad) {
  constexpr int RA = M / RB, CB = RA / RB;
  const int k = blockIdx.x;
  const int tid = threadIdx.x;
  const int g = tid & (RB - 1), ky = tid / RB;
  const size_t nat = (size_t)k * M * M + (size_t)ky * M;     // natural row ky
  const size_t ker = (size_t)k * M * M + (size_t)tid * RA;   // this thread's kernel-order run
  int badl = 0;
#pragma unroll
  for (int c = 0; c < CB; ++c)
#pragma unroll
    for (int k2 = 0; k2 < RB; ++k2) {
      const int kx = g * CB + c + RA * k2;
      if (TO_KERNEL) {
        const float x = src[nat + kx];
        if (!(x >= 0.0f) || !isfinite(x)) badl = 1;
        dst[ker + c * RB + k2] = is_sqrt ? x : sqrtf(x);
      } else {
        dst[nat + kx] = src[ker + c * RB + k2];
      }
    }
  if (badl) atomicOr(bad, 1);
}

hipError_t launch_permute_sqrt(int m, int rb, int n_pos, const float* src, int is_sqrt, float* dst, int* bad,
                               hipStream_t s) {
#define MG_PS(MM, RR) \
  if (m == MM && rb == RR) { \
    hipLaunchKernelGGL((permute_sqrt_kernel<MM, RR, 1>), dim3(n_pos), dim3(MM * RR), 0, s, n_pos, src, is_sqrt, dst, bad); \
    return hipGetLastError(); \
  }
  MG_FOR_EACH_PLAN(MG_PS)
#undef MG_PS
  return hipErrorInvalidValue;
}

hipError_t launch_unpermute_sqrt(int m, int rb, int n_pos, const float* src, float* dst, hipStream_t s) {
#define MG_US(MM, RR) \
  if (m == MM && rb == RR) { \
    hipLaunchKernelGGL((permute_sqrt_kernel<MM, RR, 0>), dim3(n_pos), dim3(MM * RR), 0, s, n_pos, src, 1, dst, nullptr); \
    return hipGetLastError(); \
  }
  MG_FOR_EACH_PLAN(MG_US)
#undef MG_US
  return hipErrorInvalidValue;
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

__global__ __launch_bounds__(256) void reduce_parts_kernel(const double* parts, int n, int nw, int take_sqrt,
                                                           double* per_pos, double* total) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    double p = 0.0;
    for (int w = 0; w < nw; ++w) p += parts[(size_t)i * MAX_WAVES + w];
    if (take_sqrt) p = sqrt(p);
    if (per_pos) per_pos[i] = p;
    s += p;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && total) *total = red[0];
}

hipError_t launch_reduce_parts(const double* parts, int n, int nw, int take_sqrt, double* per_pos, double* total,
                               hipStream_t s) {
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(1), dim3(256), 0, s, parts, n, nw, take_sqrt, per_pos, total);
  return hipGetLastError();
}


// Epoch counter for graph replays (kernels, so that a captured graph holds no memset node).
__global__ void set_counter_kernel(int* c, int v) { *c = v; }
__global__ void advance_counter_kernel(int* c) { *c += 1; }

hipError_t launch_set_counter(int* counter, int value, hipStream_t s) {
  hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(1), 0, s, counter, value);
  return hipGetLastError();
}
hipError_t launch_advance_counter(int* counter, hipStream_t s) {
  hipLaunchKernelGGL(advance_counter_kernel, dim3(1), dim3(1), 0, s, counter);
  return hipGetLastError();
}

hipError_t launch_reduce_sum(const double* x, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(256), 0, s, x, n, out);
  return hipGetLastError();
}

// Probe step (beyond the paper; simultaneous with the object step): per pixel,
// FP64 sums over the minibatch's slots in order.
// Pass 1: chunk c of PROBE_CHUNK slots; per pixel the FP64 sums of the probe
// numerator and denominator in slot order, and per chunk (one thread) the sum
// of the slots' largest |z_k|^2.  part: [chunk][3][mm], then [chunk] maxima.
__global__ __launch_bounds__(256) void probe_partial_kernel(int mm, int count, int nwaves, const float2* num,
                                                            const float* den, const float* pmax, double* part) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  const int s0 = c * PROBE_CHUNK, s1 = min(count, s0 + PROBE_CHUNK);
  const int chunks = (count + PROBE_CHUNK - 1) / PROBE_CHUNK;
  if (p < mm) {
    double nr = 0.0, ni = 0.0, dd = 0.0;
    for (int s = s0; s < s1; ++s) {
      const float2 v = num[(size_t)s * mm + p];
      nr += (double)v.x;
      ni += (double)v.y;
      dd += (double)den[(size_t)s * mm + p];
    }
    double* q = part + (size_t)c * 3 * mm;
    q[p] = nr;
    q[mm + p] = ni;
    q[2 * mm + p] = dd;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double mx = 0.0;
    for (int s = s0; s < s1; ++s) {
      float w = 0.0f;
      for (int j = 0; j < nwaves; ++j) w = fmaxf(w, pmax[(size_t)s * MAX_WAVES + j]);
      mx += (double)w;
    }
    part[(size_t)chunks * 3 * mm + c] = mx;
  }
}

// Pass 2: the chunks in order, then the probe step where the denominator is positive.
__global__ __launch_bounds__(256) void probe_apply_kernel(int mm, int chunks, double beta, const double* part,
                                                          double2* q64) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= mm) return;
  double nr = 0.0, ni = 0.0, dd = 0.0, mx = 0.0;
  for (int c = 0; c < chunks; ++c) {
    const double* q = part + (size_t)c * 3 * mm;
    nr += q[p];
    ni += q[mm + p];
    dd += q[2 * mm + p];
    mx += part[(size_t)chunks * 3 * mm + c];
  }
  dd += beta * mx;
  if (dd > 0.0) {
    double2 qq = q64[p];
    qq.x += nr / dd;
    qq.y += ni / dd;
    q64[p] = qq;
  }
}

hipError_t launch_probe_apply(int m, int count, int nwaves, const float2* num, const float* den, const float* pmax,
                              double beta, double2* q64, double* scratch, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int mm = m * m;
  const int chunks = (count + PROBE_CHUNK - 1) / PROBE_CHUNK;
  hipLaunchKernelGGL(probe_partial_kernel, dim3((mm + 255) / 256, chunks), dim3(256), 0, s, mm, count, nwaves, num,
                     den, pmax, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(probe_apply_kernel, dim3((mm + 255) / 256), dim3(256), 0, s, mm, chunks, beta, scratch, q64);
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

__global__ void fill_c64_kernel(float2* dst, size_t n, float re, float im) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = make_float2(re, im);
}

hipError_t launch_fill_c64(float2* dst, size_t n, float re, float im, hipStream_t s) {
  if (!n) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_c64_kernel, dim3(blocks), dim3(256), 0, s, dst, n, re, im);
  return hipGetLastError();
}

}  // namespace mg
