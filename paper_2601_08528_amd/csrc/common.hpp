// Device helpers shared by the HIP kernels of the library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace svf {

// Grids are capped at kMaxBlocks workgroups and walk their work in a
// grid-stride loop: a dispatch's work-items in one dimension must stay below
// 2^32, which one workgroup per row of a 200M-row table would exceed.
constexpr int64_t kMaxBlocks = 1 << 20;

constexpr int kWave = 64;
constexpr uint64_t kKeyInf = ~0ull;      // empty / padding key, flag bit set
constexpr uint32_t kEmpty = 0xffffffffu; // empty slot of an LDS id table

// ---------------------------------------------------------------------------
// Keys.  A candidate is the 64-bit word
//     [ orderable(dist) : 32 | id : 31 | expanded : 1 ]
// so unsigned comparison orders by (dist, id); the expanded flag sits in the
// lowest bit, below the id, and never decides the order of two distinct ids.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t f2ord(float f) {
  uint32_t u = __float_as_uint(f);
  if (u == 0x80000000u) u = 0u;                 // -0 and +0 are one distance
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t o) {
  uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
  return __uint_as_float(u);
}
__device__ __forceinline__ uint64_t make_key(float d, int32_t id) {
  return ((uint64_t)f2ord(d) << 32) | ((uint64_t)(uint32_t)id << 1);
}
__device__ __forceinline__ int32_t key_id(uint64_t k) {
  return k == kKeyInf ? -1 : (int32_t)(((uint32_t)k) >> 1);
}
__device__ __forceinline__ float key_dist(uint64_t k) {
  return k == kKeyInf ? __builtin_inff() : ord2f((uint32_t)(k >> 32));
}
// order-only view (flag bit forced on): distinct entries never tie
__device__ __forceinline__ uint64_t key_ord(uint64_t k) { return k | 1ull; }

// ---------------------------------------------------------------------------
// Wave primitives
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}
__device__ __forceinline__ int popc64(uint64_t m) { return __popcll(m); }
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Value of lane (lane ^ J) for a constant power of two J: a DPP quad
// permutation for 1 and 2 (a vector-ALU move, no LDS round trip), the LDS
// swizzle network for 4 to 16 (no address register), a bpermute for 32.
// Every lane of the wave must be active.  (DPP row shifts for 4 and 8, two
// moves and a select, measured slower than the swizzle in the search kernel.)
template <int J>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
  static_assert(J == 1 || J == 2 || J == 4 || J == 8 || J == 16 || J == 32, "xor_lane");
  const int x = (int)v;
  if constexpr (J == 1) {
    return (uint32_t)__builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false);   // quad [1,0,3,2]
  } else if constexpr (J == 2) {
    return (uint32_t)__builtin_amdgcn_update_dpp(x, x, 0x4E, 0xF, 0xF, false);   // quad [2,3,0,1]
  } else if constexpr (J <= 16) {
    return (uint32_t)__builtin_amdgcn_ds_swizzle(x, 0x1F | (J << 10));   // and 0x1f, xor J
  } else {
    return (uint32_t)__shfl_xor(x, 32);
  }
}
template <int J>
__device__ __forceinline__ float xor_lane_f(float v) {
  return __uint_as_float(xor_lane<J>(__float_as_uint(v)));
}
// Ascending bitonic sort of one 64-bit key per lane across the wave.
__device__ __forceinline__ uint64_t wave_sort64(uint64_t key) {
  const int lane = lane_id();
#pragma unroll
  for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      uint64_t other = __shfl_xor(key, j);
      bool up = (lane & k) == 0;
      bool low = (lane & j) == 0;
      uint64_t mn = key < other ? key : other;
      uint64_t mx = key < other ? other : key;
      key = (low == up) ? mn : mx;
    }
  }
  return key;
}

// Ordering of LDS traffic between the lanes of one wave.  A kernel whose
// workgroup is one wave uses the workgroup barrier; code run by one wave of a
// larger workgroup uses a wavefront-scope fence (a wave's LDS operations are
// performed in order; the fence keeps the compiler from moving them).
struct BlockSync {
  __device__ static __forceinline__ void sync() { __syncthreads(); }
};
struct WaveSync {
  __device__ static __forceinline__ void sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
};

// Ascending bitonic sort of n (power of two, >= 64) keys in LDS by one wave.
template <class S = BlockSync>
__device__ inline void wave_sort_lds(uint64_t* a, int n) {
  const int lane = lane_id();
  for (int k = 2; k <= n; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < n; i += kWave) {
        int p = i ^ j;
        if (p > i) {
          uint64_t x = a[i], y = a[p];
          bool up = (i & k) == 0;
          if ((x > y) == up) { a[i] = y; a[p] = x; }
        }
      }
      S::sync();
    }
  }
}

// ---------------------------------------------------------------------------
// Counter-based random numbers for entry points, from their published
// definitions: SplitMix64 (Steele, Lea, Flood 2014), j-th output from state s
// is mix(s + (j+1) * 0x9E3779B97F4A7C15); FNV-1a 64 over bytes.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t s, uint64_t j) {
  uint64_t z = s + (j + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr uint64_t kFnvBasis = 0xcbf29ce484222325ull;
constexpr uint64_t kFnvPrime = 0x100000001b3ull;

// Lemire's multiply-shift reduction of the high 32 bits into [0, n).
__device__ __forceinline__ int32_t range_reduce(uint64_t h, uint32_t n) {
  return (int32_t)(((h >> 32) * (uint64_t)n) >> 32);
}

__device__ __forceinline__ bool alive_bit(const uint32_t* bits, int32_t id) {
  return (bits[(uint32_t)id >> 5] >> (id & 31)) & 1u;
}

// Multiplicative hash into a power-of-two table.
__device__ __forceinline__ uint32_t slot_hash(uint32_t id, uint32_t mask) {
  return (id * 0x9E3779B1u) >> 7 & mask;
}

// ---------------------------------------------------------------------------
// Element conversions of the vector stores.  16-byte loads carry 4 FP32 or
// 8 FP16 / BF16 values.
// ---------------------------------------------------------------------------
struct bf16_t { uint16_t bits; };

template <typename VT> struct Elem;
template <> struct Elem<float> {
  static constexpr int kPer16B = 4;
  __device__ static __forceinline__ void unpack(const uint4& w, float* out) {
    out[0] = __uint_as_float(w.x); out[1] = __uint_as_float(w.y);
    out[2] = __uint_as_float(w.z); out[3] = __uint_as_float(w.w);
  }
  __device__ static __forceinline__ float round(float x) { return x; }
  static constexpr bool kScaled = false;
};
template <> struct Elem<__half> {
  static constexpr int kPer16B = 8;
  static constexpr bool kScaled = false;
  __device__ static __forceinline__ void unpack(const uint4& w, float* out) {
    const uint32_t v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      out[2 * i] = __half2float(__ushort_as_half((unsigned short)(v[i] & 0xffffu)));
      out[2 * i + 1] = __half2float(__ushort_as_half((unsigned short)(v[i] >> 16)));
    }
  }
  __device__ static __forceinline__ float round(float x) { return __half2float(__float2half_rn(x)); }
};
// BF16: the upper half of an FP32 word; round to nearest even on conversion.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
template <> struct Elem<bf16_t> {
  static constexpr int kPer16B = 8;
  static constexpr bool kScaled = false;
  __device__ static __forceinline__ void unpack(const uint4& w, float* out) {
    const uint32_t v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      out[2 * i] = __uint_as_float(v[i] << 16);
      out[2 * i + 1] = __uint_as_float(v[i] & 0xffff0000u);
    }
  }
  __device__ static __forceinline__ float round(float x) {
    return __uint_as_float((uint32_t)f32_to_bf16_rne(x) << 16);
  }
};


// ---------------------------------------------------------------------------
// FP8 store: OCP E4M3 codes (4 exponent bits, bias 7, 3 fraction bits, no
// infinities, largest finite 448) with one FP32 scale per vector,
// s = max|x| / 448.  A stored vector stands for s * value(code).
// ---------------------------------------------------------------------------
struct fp8_t { uint8_t bits; };

constexpr float kE4M3Max = 448.0f;

// Code of the E4M3 value nearest to v (ties to even); magnitudes beyond 448
// saturate to 448.  Built from the format's definition: below the smallest
// normal 2^-6 the grid step is 2^-9; in binade [2^E, 2^(E+1)) it is 2^(E-3).
__device__ __forceinline__ uint32_t f32_to_e4m3_sat(float v) {
  const uint32_t sign = (__float_as_uint(v) >> 24) & 0x80u;
  const float a = __builtin_fabsf(v);
  if (!(a < kE4M3Max)) return sign | 0x7Eu;
  if (a < 0.015625f) return sign | (uint32_t)__builtin_rintf(a * 512.0f);   // 0..8
  int e = __builtin_amdgcn_frexp_expf(a) - 1;                               // a in [2^e, 2^(e+1))
  uint32_t q = (uint32_t)__builtin_rintf(__builtin_ldexpf(a, 3 - e));       // 8..16
  if (q == 16u) { q = 8u; ++e; }
  uint32_t code = ((uint32_t)(e + 7) << 3) | (q - 8u);
  if (code > 0x7Eu) code = 0x7Eu;
  return sign | code;
}

// Per-vector scale from the largest magnitude (1 for an all-zero vector).
__device__ __forceinline__ float fp8_scale_of(float maxabs) {
  return maxabs > 0.0f ? __fdiv_rn(maxabs, kE4M3Max) : 1.0f;
}

template <> struct Elem<fp8_t> {
  static constexpr int kPer16B = 16;
  static constexpr bool kScaled = true;
  // gfx950 converts OCP E4M3 pairs to FP32 exactly in hardware
  __device__ static __forceinline__ void unpack(const uint4& w, float* out) {
    const uint32_t v[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)v[i], false);
      const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)v[i], true);
      out[4 * i] = lo[0]; out[4 * i + 1] = lo[1];
      out[4 * i + 2] = hi[0]; out[4 * i + 3] = hi[1];
    }
  }
  __device__ static __forceinline__ float value(uint32_t code) {
    return __builtin_amdgcn_cvt_f32_fp8((int)code, 0);
  }
};

}  // namespace svf
