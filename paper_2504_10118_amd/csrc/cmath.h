// Complex helpers and register-resident small DFTs for gfx950 kernels.
//
// Complex values are float2 (re, im).  dft<R, DIR> transforms R values held
// in registers of one thread, natural order in and out:
//     v[k] <- sum_j v[j] exp(-DIR * 2 pi i j k / R),   DIR = +1 forward, -1 inverse
// (unnormalised, the sign convention of the 2-D DFT in Section 2.1 of
// arXiv 2504.10118; the inverse uses the conjugate kernel, Appendix A).
// R is a power of two up to 32; the recursion is radix-2 decimation in time
// with compile-time twiddles, fully unrolled so that the reordering costs
// nothing but register renaming.
#pragma once
#include <hip/hip_runtime.h>

namespace mg {

// The helpers are host-callable too, so that a host build can check them.
#define MG_HD __host__ __device__ __forceinline__

MG_HD float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
MG_HD float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
MG_HD float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
MG_HD float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
MG_HD float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// a * exp(-DIR * i pi / 2): forward multiplies by -i, inverse by +i.
template <int DIR>
MG_HD float2 mul_quarter(float2 a) {
  return DIR > 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

// a * exp(-DIR * 2 pi i j / 16) for a compile-time j in [0, 8).
template <int J, int DIR>
MG_HD float2 mul_w16(float2 a) {
  constexpr float C1 = 0.92387953251128675613f;   // cos(pi/8)
  constexpr float S1 = 0.38268343236508977173f;   // sin(pi/8)
  constexpr float H = 0.70710678118654752440f;    // cos(pi/4)
  constexpr float s = DIR > 0 ? -1.0f : 1.0f;     // sign of the sine part
  if constexpr (J == 0) {
    return a;
  } else if constexpr (J == 4) {
    return mul_quarter<DIR>(a);
  } else if constexpr (J == 2) {
    // (c + i s c) with c = H
    return make_float2(H * (a.x - s * a.y), H * (a.y + s * a.x));
  } else if constexpr (J == 6) {
    // (-c + i s c)
    return make_float2(H * (-a.x - s * a.y), H * (-a.y + s * a.x));
  } else {
    constexpr float c = (J == 1) ? C1 : (J == 3) ? S1 : (J == 5) ? -S1 : -C1;
    constexpr float sn = (J == 1) ? S1 : (J == 3) ? C1 : (J == 5) ? C1 : S1;
    // a * (c + i s sn)
    return make_float2(a.x * c - a.y * (s * sn), a.x * (s * sn) + a.y * c);
  }
}

// a * exp(-DIR * 2 pi i j / 32) for a compile-time j in [0, 16): even j reduce
// to the 16-point twiddles; odd j use cos and sin of (2j + 1) pi / 32 folded
// onto the first octant by the symmetries of the circle.
template <int J, int DIR>
MG_HD float2 mul_w32(float2 a) {
  if constexpr (J % 2 == 0) {
    return mul_w16<J / 2, DIR>(a);
  } else {
    constexpr float C1 = 0.98078528040323044913f;   // cos(pi/16)
    constexpr float S1 = 0.19509032201612826785f;   // sin(pi/16)
    constexpr float C3 = 0.83146961230254523708f;   // cos(3 pi/16)
    constexpr float S3 = 0.55557023301960222474f;   // sin(3 pi/16)
    constexpr float s = DIR > 0 ? -1.0f : 1.0f;
    constexpr float c = (J == 1) ? C1 : (J == 3) ? C3 : (J == 5) ? S3 : (J == 7) ? S1
                      : (J == 9) ? -S1 : (J == 11) ? -S3 : (J == 13) ? -C3 : -C1;
    constexpr float sn = (J == 1) ? S1 : (J == 3) ? S3 : (J == 5) ? C3 : (J == 7) ? C1
                       : (J == 9) ? C1 : (J == 11) ? C3 : (J == 13) ? S3 : S1;
    return make_float2(a.x * c - a.y * (s * sn), a.x * (s * sn) + a.y * c);
  }
}

// a * W_32^j for j known after unrolling (the switch folds away)
template <int DIR>
MG_HD float2 mul_w32_at(int j, float2 a) {
  switch (j) {
    case 0: return a;
    case 1: return mul_w32<1, DIR>(a);
    case 2: return mul_w32<2, DIR>(a);
    case 3: return mul_w32<3, DIR>(a);
    case 4: return mul_w32<4, DIR>(a);
    case 5: return mul_w32<5, DIR>(a);
    case 6: return mul_w32<6, DIR>(a);
    case 7: return mul_w32<7, DIR>(a);
    case 8: return mul_w32<8, DIR>(a);
    case 9: return mul_w32<9, DIR>(a);
    case 10: return mul_w32<10, DIR>(a);
    case 11: return mul_w32<11, DIR>(a);
    case 12: return mul_w32<12, DIR>(a);
    case 13: return mul_w32<13, DIR>(a);
    case 14: return mul_w32<14, DIR>(a);
    default: return mul_w32<15, DIR>(a);
  }
}

template <int R, int DIR>
MG_HD void dft(float2* v) {
  static_assert(R >= 1 && R <= 32 && (R & (R - 1)) == 0, "dft: R must be a power of two up to 32");
  if constexpr (R == 1) {
    return;
  } else if constexpr (R == 2) {
    float2 t = v[0];
    v[0] = cadd(t, v[1]);
    v[1] = csub(t, v[1]);
  } else if constexpr (R == 4) {
    float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    float2 t2 = cadd(v[1], v[3]), t3 = mul_quarter<DIR>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  } else {
    constexpr int H = R / 2;
    float2 e[H], o[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
      e[i] = v[2 * i];
      o[i] = v[2 * i + 1];
    }
    dft<H, DIR>(e);
    dft<H, DIR>(o);
    // twiddle W_R^k = W_32^(k * 32 / R)
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const float2 t = mul_w32_at<DIR>(k * (32 / R), o[k]);
      v[k] = cadd(e[k], t);
      v[k + H] = csub(e[k], t);
    }
  }
}

}  // namespace mg

namespace mg {

// Value of the lane whose id differs from this lane's in bit MASK (a power of
// two below 64).  Masks 1 and 2 are DPP quad_perm, 8 is DPP row_ror:8.  The
// others come in two forms:
//   VALU = true (VF: a bit mask of the distances 4, 16, 32 that take this form):
//     VALU cross-lane operations only, for latency-bound kernels
//     with few waves per SIMD (the LDS-pipe round trips of the other form sit
//     on their critical path): 4 selects between row_ror:12 and row_ror:4
//     (row_ror:N gives lane l the value of lane l - N of its 16-lane row, mod
//     16: N = 12 reads lane l + 4, the partner of lanes with bit 2 clear, N = 4
//     reads lane l - 4, the partner of the others); 16 and 32 use gfx950's
//     v_permlane16_swap / v_permlane32_swap of the value with itself, which give
//     (row 0, row 0, row 2, row 2) and (row 1, row 1, row 3, row 3) for 16-lane
//     rows (halves 0, 0 and 1, 1 for 32), so the partner's value is the first
//     result in odd rows (halves) and the second in even ones;
//   VALU = false: ds_swizzle (4, 16) and ds_bpermute (32) in the LDS pipe, which
//     cost no VALU issue slots where enough waves hide their latency.
constexpr int XOR_ALL_VALU = 4 | 16 | 32;
template <int MASK, int VF = XOR_ALL_VALU>
__device__ __forceinline__ int xor_lane(int v) {
  constexpr bool VALU = (VF & MASK) != 0;
  static_assert(MASK > 0 && MASK < 64 && (MASK & (MASK - 1)) == 0, "power of two below 64");
  if constexpr (MASK == 1) {
    return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  } else if constexpr (MASK == 2) {
    return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  } else if constexpr (MASK == 8) {
    return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);  // row_ror:8
  } else if constexpr (!VALU) {
    if constexpr (MASK == 4) return __builtin_amdgcn_ds_swizzle(v, 0x101F);    // and 0x1f, xor 4
    else if constexpr (MASK == 16) return __builtin_amdgcn_ds_swizzle(v, 0x401F);  // and 0x1f, xor 16
    else return __shfl_xor(v, MASK);
  } else if constexpr (MASK == 4) {
    const int r4 = __builtin_amdgcn_update_dpp(0, v, 0x124, 0xF, 0xF, false);    // row_ror:4
    const int r12 = __builtin_amdgcn_update_dpp(0, v, 0x12C, 0xF, 0xF, false);   // row_ror:12
    return (__lane_id() & 4) ? r4 : r12;
  } else if constexpr (MASK == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (__lane_id() & 16) ? (int)r[0] : (int)r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (__lane_id() & 32) ? (int)r[0] : (int)r[1];
  }
}

template <int MASK, int VF = XOR_ALL_VALU>
__device__ __forceinline__ double xor_lane(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = xor_lane<MASK, VF>((int)(b & 0xffffffffll));
  const int hi = xor_lane<MASK, VF>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int MASK, int VF = XOR_ALL_VALU>
__device__ __forceinline__ double2 xor_lane(double2 v) {
  return make_double2(xor_lane<MASK, VF>(v.x), xor_lane<MASK, VF>(v.y));
}

// Runtime mask dispatch (the mask is uniform and comes from a small set).
template <int VF = XOR_ALL_VALU>
__device__ __forceinline__ double2 xor_lane_rt(double2 v, int mask) {
  switch (mask) {
    case 1: return xor_lane<1, VF>(v);
    case 2: return xor_lane<2, VF>(v);
    case 4: return xor_lane<4, VF>(v);
    case 8: return xor_lane<8, VF>(v);
    case 16: return xor_lane<16, VF>(v);
    default: return xor_lane<32, VF>(v);
  }
}

}  // namespace mg

namespace mg {

// Raw buffer access: a scalar 128-bit resource (base, size in bytes), a
// 32-bit per-lane byte offset and a scalar byte offset.  Loads outside the
// resource return zero and stores there are dropped.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kBufferFlags = 0x00020000;   // gfx9 descriptor word 3 (32-bit raw data)

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufferFlags);
}
__device__ __forceinline__ float2 bload2(rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ float4 bload4(rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
// Cache-policy bits of gfx950 vector memory instructions: SC1 alone gives a
// store device scope, i.e. written through this XCD's L2.
constexpr int kPolicyDeviceScope = 0x10;

// Load with a cache policy fixed at compile time; with kPolicyDeviceScope it
// reads the value at device scope, coherent with device-scope stores that
// workgroups on other XCDs made earlier in the same launch.
template <int POL>
__device__ __forceinline__ float2 bload2p(rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, POL));
}

__device__ __forceinline__ void bstore2(rsrc_t r, float2 v, int voff, int soff) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
}
// Store for data the next kernel reads on other XCDs (the staged updates): with
// device scope it leaves no dirty L2 lines to be written back when the kernel
// ends (measured: -1.6 us per 256-pattern launch at m = 64, -1 us at m = 128),
// but in launches of many workgroups per CU the write-through costs more than
// the write-back it saves (+6 % on 16 k-workgroup launches).
__device__ __forceinline__ void bstore2_device(rsrc_t r, float2 v, int voff, int soff) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, kPolicyDeviceScope);
}
__device__ __forceinline__ void bstore2_stage(rsrc_t r, float2 v, int voff, int soff, bool device_scope) {
  if (device_scope) bstore2_device(r, v, voff, soff);
  else bstore2(r, v, voff, soff);
}

}  // namespace mg
