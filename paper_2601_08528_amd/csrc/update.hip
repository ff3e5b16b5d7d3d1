// Index maintenance kernels: seed graph, insertion (Sec. 5.1) and deletion
// with localized repair and consolidation (Sec. 5.2).
//
// Rank-based candidate reordering (Sec. 5.1) is computed without distance
// evaluations.  For a vertex with candidates c_0..c_{m-1} in (d,id) order, the
// wave builds an LDS map id -> position, scans the neighbour rows of every
// candidate c_j with coalesced loads, and for each row entry that is a later
// candidate c_i (i > j) adds one to its detour count with an LDS atomic.  The
// R kept candidates are those of smallest (count, position): a histogram of
// the counts gives the threshold count tau, then one ordered ballot pass keeps
// every candidate below tau and the first ones equal to tau, and writes them
// in position order, which is (d,id) order.
//
// Every batch reads one snapshot and writes staged rows; a commit kernel
// copies them into the graph afterwards, so the result never depends on the
// order in which waves run.
#include <algorithm>
#include <type_traits>

#include "common.hpp"
#include "kernels.hpp"
#include "wave_ops.hpp"

namespace svf {

namespace {

__device__ __forceinline__ int wave_incl_scan(int x) {
  const int lane = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int t = __shfl_up(x, o);
    if (lane >= o) x += t;
  }
  return x;
}

struct RowSource {
  const int32_t* graph;
  const int32_t* fwd;
  int32_t n_old;
  int R;
  __device__ __forceinline__ const int32_t* row(int32_t id) const {
    return id < n_old ? graph + (int64_t)id * R : fwd + (int64_t)(id - n_old) * R;
  }
};

// Candidate id -> position table of the prune: S slots (a power of two, at
// least four per candidate, so that ids sit close to their home slots) of
// ids with linear probing, each with its candidate's 16-bit position in a
// second array, followed by a copy of the first kProbeMax slots of both so
// that a lookup reads consecutive slots without wrapping.  dmax is the largest
// distance of an inserted id from its home slot; a lookup that reads the
// dmax + 1 slots from the home slot finds any inserted id.  A lookup reads
// 4-byte ids and fetches a position only on a hit.  A free slot holds
// kFree, which is neither an id nor the -1 that pads rows, so an entry read
// from a row never matches a free slot.
constexpr int kProbeMax = 8;
constexpr uint32_t kFree = 0xfffffffeu;
// The positions come first, at the start of the kernel's LDS, so that the
// address of a hit's position is one shift-and-add of its slot.
struct PruneLds {
  uint16_t* mval;   // S + kProbeMax positions
  uint32_t* mkey;   // S + kProbeMax slots (kFree when free)
  uint32_t* cnt;    // cap
  uint32_t* hist;   // cap + 1
  uint32_t* dmax;   // 1
  int S;
};

// Byte offset from the home slot's position to the position of candidate id
// e (-1 if e is not a candidate, -1 included) when the table's largest
// displacement is below N: a fixed read of the N slots from the home slot,
// with no data-dependent branch.  The offsets are constants of the unrolled
// compare chain.
template <int N>
__device__ __forceinline__ int tab_off(const PruneLds& s, uint32_t home, int32_t e) {
  uint32_t w[N];
#pragma unroll
  for (int d = 0; d < N; ++d) w[d] = s.mkey[home + d];
  int off = -1;
#pragma unroll
  for (int d = 0; d < N; ++d)
    if (w[d] == (uint32_t)e) off = 2 * d;
  return off;
}
__device__ __forceinline__ int tab_pos(const PruneLds& s, uint32_t home, int off) {
  return *reinterpret_cast<const uint16_t*>(reinterpret_cast<const unsigned char*>(s.mval + home) +
                                            off);
}
// The same with any displacement (a probe loop that stops at an empty slot).
__device__ __forceinline__ int tab_find_loop(const PruneLds& s, uint32_t home, int32_t e,
                                             uint32_t mask) {
  if (e < 0) return -1;
  uint32_t sl = home;
  for (;;) {
    const uint32_t k = s.mkey[sl];
    if (k == (uint32_t)e) return (int)s.mval[sl];
    if (k == kFree) return -1;
    sl = (sl + 1) & mask;
  }
}

// Home slot of an id in the prune's table (S = 2^sbits slots): bits 7 and up
// of a multiplicative hash of the id's low 24 bits, on the full-rate 24-bit
// multiplier (a 32-bit multiply issues at a quarter of the rate).  Ids equal
// in their low 24 bits share a home slot; that only lengthens probes.
__device__ __forceinline__ uint32_t prune_hash(uint32_t id, uint32_t sbits) {
  return __builtin_amdgcn_ubfe(__umul24(id, 0x9E3779u), 7u, sbits);
}

// Fourth word of a raw (unformatted, unswizzled) buffer resource on gfx9
// targets: 32-bit data format, so that a dword load returns the dword.  A row
// read through a resource takes its base from two scalar registers and the
// lane's byte offset from a vector register, with no address arithmetic per
// row; offsets past the resource's size return 0 instead of reading memory.
constexpr int kRawBufferWord3 = 0x00020000;

__device__ __forceinline__ int pow2_at_least(int x, int lo) {
  int p = lo;
  while (p < x) p <<= 1;
  return p;
}

// Calls f with the number of slots a lookup reads as a compile-time constant
// (1 .. kProbeMax), or 0 for the probe loop when the displacement is larger.
template <class F>
__device__ __forceinline__ void probe_by_slots(int nd, F&& f) {
  switch (nd) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    default: f(std::integral_constant<int, 0>{}); break;
  }
}

// Rank-based reordering of the m sorted candidate keys in LDS; writes R ids
// and distances (INVALID / +inf padded) to out.
__device__ void prune_core(const uint64_t* keys, int m, const RowSource& rs, int R, PruneLds& s,
                           int32_t* __restrict__ out_ids, float* __restrict__ out_d) {
  const int lane = lane_id();
  int tau = 0, need = 0;
  const bool full = m > R;
  if (full) {
    // S is a power of two >= 64 and the slots start 16-byte aligned
    for (int i = 4 * lane; i < s.S; i += 4 * kWave)
      *reinterpret_cast<uint4*>(s.mkey + i) = make_uint4(kFree, kFree, kFree, kFree);
    for (int i = lane; i <= m; i += kWave) { s.hist[i] = 0; if (i < m) s.cnt[i] = 0; }
    if (lane == 0) *s.dmax = 0;
    __syncthreads();
    const uint32_t mask = (uint32_t)s.S - 1u;
    const uint32_t sbits = (uint32_t)__builtin_ctz((uint32_t)s.S);
    for (int i = lane; i < m; i += kWave) {
      const uint32_t id = (uint32_t)key_id(keys[i]);
      uint32_t sl = prune_hash(id, sbits), d = 0;
      while (atomicCAS(&s.mkey[sl], kFree, id) != kFree) {
        sl = (sl + 1) & mask;
        ++d;
      }
      s.mval[sl] = (uint16_t)i;
      atomicMax(s.dmax, d);
    }
    __syncthreads();
    for (int i = lane; i < kProbeMax; i += kWave) {
      s.mkey[s.S + i] = s.mkey[i];
      s.mval[s.S + i] = s.mval[i];
    }
    const int nd = uniform((int)*s.dmax) + 1;   // slots a lookup reads
    __syncthreads();
    // detour counts: entry r of row(c_j) naming c_i with i > j.  The counts
    // are sums, so the order in which entries are probed does not matter.
    if (R > 32 && R <= kWave) {
      // One whole row per step, 8 rows per pass: lane r reads entry r of row
      // j.  Row addresses are computed 64 rows at a time (lane l holds the
      // byte address of row g + l) and read out lane by lane into a buffer
      // resource per row, so each load is a scalar base plus the lane's byte
      // offset.  Every load is issued, with no branch: lanes past the row
      // re-read its last entry and rows past m re-read row 0; neither is
      // probed.  The rows of the next pass are requested before the entries
      // of this one are probed (after the last pass, 8 reads of row 0 that
      // are never used), so that the probes run while those reads are in
      // flight.
      constexpr int kRowSteps = 8;
      const bool lane_on = lane < R;
      const uint32_t lbyte = 4u * (uint32_t)(lane_on ? lane : R - 1);
      uint32_t ra_lo = 0, ra_hi = 0;
      auto address_rows = [&](int g) {
        const int j = g + lane < m ? g + lane : 0;
        const uint64_t ra = (uint64_t)(uintptr_t)rs.row(key_id(keys[j]));
        ra_lo = (uint32_t)ra;
        ra_hi = (uint32_t)(ra >> 32);
      };
      auto load_pass = [&](int j0, int32_t (&e)[kRowSteps]) {
        const int l0 = j0 & (kWave - 1);
#pragma unroll
        for (int u = 0; u < kRowSteps; ++u) {
          const uint64_t b =
              ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(ra_hi, l0 + u) << 32) |
              (uint32_t)__builtin_amdgcn_readlane(ra_lo, l0 + u);
          const __amdgpu_buffer_rsrc_t row = __builtin_amdgcn_make_buffer_rsrc(
              reinterpret_cast<void*>(b), (short)0, 4 * R, kRawBufferWord3);
          e[u] = __builtin_amdgcn_raw_buffer_load_b32(row, lbyte, 0, 0);
        }
      };
      int32_t e[kRowSteps], en[kRowSteps];
      address_rows(0);
      load_pass(0, e);
      for (int j0 = 0; j0 < m; j0 += kRowSteps) {
        const int jn = j0 + kRowSteps;
        if ((jn & (kWave - 1)) == 0) address_rows(jn);
        load_pass(jn, en);
        auto count = [&](auto nslots) {
#pragma unroll
          for (int u = 0; u < kRowSteps; ++u) {
            constexpr int N = decltype(nslots)::value;
            if (j0 + u >= m) break;          // rows past the list (last pass only)
            const uint32_t h = prune_hash((uint32_t)e[u], sbits);
            const int jt = j0 + u;
            if constexpr (N > 0) {
              const int off = tab_off<N>(s, h, e[u]);
              if (off >= 0) {
                const int i = tab_pos(s, h, off);
                if (i > jt) atomicAdd(&s.cnt[i], 1u);
              }
            } else {
              const int i = tab_find_loop(s, h, e[u], mask);
              if (i > jt) atomicAdd(&s.cnt[i], 1u);
            }
          }
        };
        if (lane_on) probe_by_slots(nd, count);
#pragma unroll
        for (int u = 0; u < kRowSteps; ++u) e[u] = en[u];
      }
    } else {
      // Any degree: entry t = j * R + r goes to lane t % 64; each lane loads
      // kRowSteps entries (rows of different candidates) before it probes
      // any, so that many row reads are in flight per wave.
      constexpr int kRowSteps = 8;
      const int total = m * R;
      int j0 = lane / R, r0 = lane - (lane / R) * R;   // (j, r) of entry t0 + lane
      for (int t0 = 0; t0 < total; t0 += kWave * kRowSteps) {
        int32_t e[kRowSteps];
        int jj[kRowSteps];
        int j = j0, r = r0;
#pragma unroll
        for (int u = 0; u < kRowSteps; ++u) {
          jj[u] = j;
          e[u] = t0 + u * kWave + lane < total ? rs.row(key_id(keys[j]))[r] : -1;
          r += kWave;
          while (r >= R) { r -= R; ++j; }
        }
        j0 = j;
        r0 = r;
        auto count = [&](auto nslots) {
#pragma unroll
          for (int u = 0; u < kRowSteps; ++u) {
            constexpr int N = decltype(nslots)::value;
            const uint32_t h = prune_hash((uint32_t)e[u], sbits);
            if constexpr (N > 0) {
              const int off = tab_off<N>(s, h, e[u]);
              if (off >= 0) {
                const int i = tab_pos(s, h, off);
                if (i > jj[u]) atomicAdd(&s.cnt[i], 1u);
              }
            } else {
              const int i = tab_find_loop(s, h, e[u], mask);
              if (i > jj[u]) atomicAdd(&s.cnt[i], 1u);
            }
          }
        };
        probe_by_slots(nd, count);
      }
    }
    __syncthreads();
    for (int i = lane; i < m; i += kWave) atomicAdd(&s.hist[s.cnt[i]], 1u);
    __syncthreads();
    // tau: smallest count value whose cumulative frequency reaches R
    int run = 0;
    tau = -1;
    for (int c0 = 0; c0 < m && tau < 0; c0 += kWave) {
      const int h = c0 + lane < m ? (int)s.hist[c0 + lane] : 0;
      const int incl = wave_incl_scan(h);
      const uint64_t hit = ballot(run + incl >= R);
      if (hit) {
        const int l = __ffsll((unsigned long long)hit) - 1;
        const int incl_l = __shfl(incl, l);
        const int h_l = __shfl(h, l);
        tau = c0 + l;
        need = R - (run + incl_l - h_l);
      }
      run += __shfl(incl, kWave - 1);
    }
  }
  // keep: all below tau, then the first `need` equal to tau, in position order
  int outpos = 0, eq_seen = 0;
  for (int c0 = 0; c0 < m; c0 += kWave) {
    const int i = c0 + lane;
    const bool on = i < m;
    bool sel = on;
    if (full) {
      const int c = on ? (int)s.cnt[i] : 0x7fffffff;
      const bool eq = on && c == tau;
      const uint64_t eb = ballot(eq);
      sel = on && (c < tau || (eq && eq_seen + lanes_below(eb) < need));
      eq_seen += popc64(eb);
    }
    const uint64_t sb = ballot(sel);
    if (sel) {
      const int p = outpos + lanes_below(sb);
      const uint64_t k = keys[i];
      out_ids[p] = key_id(k);
      out_d[p] = key_dist(k);
    }
    outpos += popc64(sb);
  }
  for (int i = outpos + lane; i < R; i += kWave) { out_ids[i] = -1; out_d[i] = __builtin_inff(); }
  __syncthreads();
}

// LDS of the prune for lists of up to cap candidates, at the start of the
// kernel's LDS: positions, slots, counts, histogram, displacement; its size is
// a multiple of 16 bytes so that what follows stays aligned.
__host__ __device__ inline int prune_table_slots(int cap) {
  int S = 64;
  while (S < 4 * cap) S <<= 1;
  return S;
}
__host__ __device__ inline int prune_scratch_bytes_of(int cap) {
  const int S = prune_table_slots(cap);
  return ((S + kProbeMax) * 6 + cap * 4 + (cap + 1) * 4 + 4 + 15) / 16 * 16;
}
__device__ __forceinline__ PruneLds carve_prune_lds(unsigned char* smem, int cap) {
  PruneLds s;
  s.S = prune_table_slots(cap);
  s.mval = reinterpret_cast<uint16_t*>(smem);
  s.mkey = reinterpret_cast<uint32_t*>(smem + 2 * (s.S + kProbeMax));
  s.cnt = s.mkey + s.S + kProbeMax;
  s.hist = s.cnt + cap;
  s.dmax = s.hist + cap + 1;
  return s;
}
size_t prune_scratch_bytes(int cap) { return (size_t)prune_scratch_bytes_of(cap); }
// LDS in front of the reverse-edge pool: the prune table, or while the pool is
// merged, the merge buffers (cap + one wave of keys).
__host__ __device__ inline int reverse_table_bytes(int cap) {
  const int t = prune_scratch_bytes_of(cap), mb = (cap + kWave) * 8;
  return t > mb ? t : (mb + 15) / 16 * 16;
}

// Number of non-padding keys in a sorted LDS list of n keys.
__device__ __forceinline__ int count_keys(const uint64_t* a, int n) {
  int m = 0;
  for (int c0 = 0; c0 < n; c0 += kWave) {
    const int i = c0 + lane_id();
    m += popc64(ballot(i < n && a[i] != kKeyInf));
  }
  return m;
}

}  // namespace

// ---------------------------------------------------------------------------
__global__ void fill_u32_kernel(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
hipError_t launch_fill_u32(void* p, int64_t n, uint32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, st,
                     static_cast<uint32_t*>(p), n, v);
  return hipGetLastError();
}

// FP32 rows -> FP16 / BF16 rows (round to nearest even).
__global__ void store_lowp_kernel(const float* __restrict__ src, uint16_t* __restrict__ dst,
                                  int64_t n, int precision) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float x = src[i];
    dst[i] = precision == 1 ? __half_as_ushort(__float2half_rn(x)) : f32_to_bf16_rne(x);
  }
}
// FP32 rows -> FP8 rows, one wave per row: the scale from the row's largest
// magnitude, then the E4M3 code of each x / s; the row's tail up to lp_stride
// is zero.
__global__ __launch_bounds__(256) void store_fp8_kernel(const float* __restrict__ src,
                                                        int64_t stride, int dim,
                                                        uint8_t* __restrict__ dst,
                                                        int64_t lp_stride, float* __restrict__ scale,
                                                        int64_t nrows) {
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  const int lane = lane_id();
  for (int64_t r = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; r < nrows;
       r += waves) {
    const float* x = src + r * stride;
    float m = 0.0f;
    for (int i = lane; i < dim; i += kWave) m = __builtin_fmaxf(m, __builtin_fabsf(x[i]));
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) m = __builtin_fmaxf(m, __shfl_xor(m, o));
    const float s = fp8_scale_of(m);
    uint8_t* y = dst + r * lp_stride;
    for (int i = lane; i < lp_stride; i += kWave)
      y[i] = i < dim ? (uint8_t)f32_to_e4m3_sat(__fdiv_rn(x[i], s)) : (uint8_t)0;
    if (lane == 0) scale[r] = s;
  }
}

hipError_t launch_store_lowp(const float* src, int64_t stride, int dim, void* veclp,
                             int64_t lp_stride, float* vscale, int64_t row0, int64_t nrows,
                             int precision, hipStream_t st) {
  if (nrows <= 0 || precision == 0) return hipSuccess;
  if (precision == 3) {
    const int64_t blocks = std::min<int64_t>((nrows + 3) / 4, kMaxBlocks);
    hipLaunchKernelGGL(store_fp8_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, stride, dim,
                       static_cast<uint8_t*>(veclp) + row0 * lp_stride, lp_stride, vscale + row0,
                       nrows);
    return hipGetLastError();
  }
  const int64_t n = nrows * stride;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(store_lowp_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src,
                     static_cast<uint16_t*>(veclp) + row0 * stride, n, precision);
  return hipGetLastError();
}

// Scales of the vectors a row names, stored beside the row (FP8 traversal):
// one thread per row entry, over listed rows or a range of rows.
__global__ void row_scales_kernel(const int32_t* __restrict__ graph, int R,
                                  const int32_t* __restrict__ list, int64_t lo, int64_t n,
                                  const float* __restrict__ vscale, float* __restrict__ nscale) {
  const int64_t total = n * R;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = i / R, r = i - k * R;
    const int64_t v = list ? (int64_t)list[k] : lo + k;
    const int32_t u = graph[v * R + r];
    nscale[v * R + r] = u >= 0 ? vscale[u] : 0.0f;
  }
}
hipError_t launch_row_scales(const int32_t* graph, int R, const int32_t* list, int64_t lo, int64_t n,
                             const float* vscale, float* nscale, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n * R + 255) / 256, kMaxBlocks);
  hipLaunchKernelGGL(row_scales_kernel, dim3((unsigned)blocks), dim3(256), 0, st, graph, R, list, lo,
                     n, vscale, nscale);
  return hipGetLastError();
}

__global__ void set_alive_kernel(uint32_t* alive, int64_t lo, int64_t hi) {
  const int64_t i = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < hi) atomicOr(&alive[i >> 5], 1u << (i & 31));
}
hipError_t launch_set_alive(uint32_t* alive, int64_t lo, int64_t hi, hipStream_t st) {
  if (hi <= lo) return hipSuccess;
  hipLaunchKernelGGL(set_alive_kernel, dim3((unsigned)((hi - lo + 255) / 256)), dim3(256), 0, st,
                     alive, lo, hi);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Seed graph: with every neighbour list empty all detour counts are 0, so each
// seed vertex keeps its R nearest other seed vertices.
template <int NC>
__global__ __launch_bounds__(64) void seed_kernel(const float* __restrict__ vec32, int64_t stride,
                                                  int dim, int metric, int s0, int R,
                                                  int32_t* graph, float* edge_d) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int v = blockIdx.x;
  const int lane = lane_id();
  const int n = pow2_at_least(s0, 64);
  uint64_t* keys = reinterpret_cast<uint64_t*>(smem);
  int32_t* cid = reinterpret_cast<int32_t*>(keys + n);
  QuerySlice<float, NC> q;
  q.load(vec32 + (int64_t)v * stride, dim, lane % QuerySlice<float, NC>::kLanesPerVec);
  for (int c0 = 0; c0 < n; c0 += kWave) {
    const int u = c0 + lane;
    const bool on = u < s0 && u != v;
    const uint64_t ob = ballot(on);
    if (on) cid[lanes_below(ob)] = u;
    __syncthreads();
    const uint64_t k = gather_keys<float, NC>(q, vec32, stride, cid, popc64(ob), metric);
    keys[c0 + lane] = k;
    __syncthreads();
  }
  wave_sort_lds(keys, n);
  for (int r = lane; r < R; r += kWave) {
    const uint64_t k = r < s0 - 1 ? keys[r] : kKeyInf;
    graph[(int64_t)v * R + r] = key_id(k);
    edge_d[(int64_t)v * R + r] = key_dist(k);
  }
}
hipError_t launch_seed(const float* vec32, int64_t stride, int dim, int metric, int s0, int R,
                       int32_t* graph, float* edge_d, hipStream_t st) {
  if (s0 <= 0) return hipSuccess;
  int n = 64;
  while (n < s0) n <<= 1;
  const size_t lds = (size_t)n * 8 + kWave * 4;
  const int chunks = (int)((stride + 127) / 128);
  dim3 g(s0), b(kWave);
  switch (chunks <= 1 ? 1 : chunks <= 2 ? 2 : chunks <= 4 ? 4 : 8) {
    case 1: hipLaunchKernelGGL(seed_kernel<1>, g, b, lds, st, vec32, stride, dim, metric, s0, R, graph, edge_d); break;
    case 2: hipLaunchKernelGGL(seed_kernel<2>, g, b, lds, st, vec32, stride, dim, metric, s0, R, graph, edge_d); break;
    case 4: hipLaunchKernelGGL(seed_kernel<4>, g, b, lds, st, vec32, stride, dim, metric, s0, R, graph, edge_d); break;
    default: hipLaunchKernelGGL(seed_kernel<8>, g, b, lds, st, vec32, stride, dim, metric, s0, R, graph, edge_d); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Prune of candidate lists held in global memory (forward rows of a batch,
// repaired rows).
__global__ __launch_bounds__(64) void prune_lists_kernel(PruneArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int li = blockIdx.x;
  if (li >= a.nlists) return;
  if (a.skip && a.skip[li] < 0) return;
  const int lane = lane_id();
  const int cap = a.cap < a.cstride ? a.cap : a.cstride;
  PruneLds s = carve_prune_lds(smem, cap);
  uint64_t* keys = reinterpret_cast<uint64_t*>(smem + prune_scratch_bytes_of(cap));
  const uint64_t* src = a.cand + (int64_t)li * a.cstride;
  for (int i = lane; i < cap; i += kWave) keys[i] = src[i];
  __syncthreads();
  const int m = count_keys(keys, cap);
  RowSource rs{a.graph, a.fwd, a.n_old, a.R};
  prune_core(keys, m, rs, a.R, s, a.out_ids + (int64_t)li * a.R, a.out_d + (int64_t)li * a.R);
}
size_t prune_lds_bytes(int cap) { return (size_t)cap * 8 + prune_scratch_bytes(cap); }
hipError_t launch_prune_lists(const PruneArgs& a, hipStream_t st) {
  if (a.nlists <= 0) return hipSuccess;
  const int cap = a.cap < a.cstride ? a.cap : a.cstride;
  hipLaunchKernelGGL(prune_lists_kernel, dim3(a.nlists), dim3(kWave), prune_lds_bytes(cap), st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reverse edges (Sec. 5.1): group (target, new vertex, distance) by target.
__global__ void reverse_count_kernel(ReverseArgs a) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)a.b * a.R) return;
  const int32_t t = a.fwd_ids[i];
  if (t < 0 || (a.tmask && !((a.tmask[t >> 5] >> (t & 31)) & 1u))) return;
  if (atomicAdd(&a.tcount[t], 1) == 0) {
    const int k = atomicAdd(a.n_targets, 1);
    a.tlist[k] = t;
    a.tidx[t] = k;
  }
}
hipError_t launch_reverse_count(const ReverseArgs& a, hipStream_t st) {
  const int64_t n = (int64_t)a.b * a.R;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(reverse_count_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

// Exclusive scan of the per-target counts: each 256-thread block scans 1024
// targets and records its total; one block scans the totals; a last pass adds
// the block offsets and resets the scatter cursors.
constexpr int kScanBlock = 1024;
__device__ __forceinline__ int block_excl_scan_256(int v, int* sh, int* total) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  int incl = wave_incl_scan(v);
  if (lane == 63) sh[wv] = incl;
  __syncthreads();
  int base = 0;
  for (int i = 0; i < wv; ++i) base += sh[i];
  *total = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return base + incl - v;
}
__global__ __launch_bounds__(256) void scan_blocks_kernel(ReverseArgs a, int n, int32_t* bsum) {
  __shared__ int sh[4];
  const int b0 = blockIdx.x * kScanBlock + threadIdx.x * 4;
  int v[4], s = 0;
  for (int i = 0; i < 4; ++i) {
    v[i] = b0 + i < n ? a.tcount[a.tlist[b0 + i]] : 0;
    s += v[i];
  }
  int total;
  int e = block_excl_scan_256(s, sh, &total);
  for (int i = 0; i < 4; ++i) {
    if (b0 + i < n) a.off[b0 + i] = e;
    e += v[i];
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}
__global__ __launch_bounds__(256) void scan_totals_kernel(int32_t* bsum, int nb) {
  __shared__ int sh[4];
  int run = 0;
  for (int c0 = 0; c0 < nb; c0 += 256) {
    const int i = c0 + threadIdx.x;
    const int v = i < nb ? bsum[i] : 0;
    int total;
    const int e = block_excl_scan_256(v, sh, &total);
    if (i < nb) bsum[i] = run + e;
    run += total;
  }
  if (threadIdx.x == 0) bsum[nb] = run;
}
__global__ __launch_bounds__(256) void scan_add_kernel(ReverseArgs a, int n, const int32_t* bsum, int nb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    a.off[i] += bsum[i / kScanBlock];
    a.cursor[i] = 0;
  }
  if (i == 0) a.off[n] = bsum[nb];
}
__global__ void reverse_scatter_kernel(ReverseArgs a) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)a.b * a.R) return;
  const int32_t t = a.fwd_ids[i];
  if (t < 0 || (a.tmask && !((a.tmask[t >> 5] >> (t & 31)) & 1u))) return;
  const int k = a.tidx[t];
  const int pos = a.off[k] + atomicAdd(&a.cursor[k], 1);
  a.inc[pos] = make_key(a.fwd_d[i], a.n0 + (int32_t)(i / a.R));
}
hipError_t launch_reverse_scan_scatter(const ReverseArgs& a, int n_targets, hipStream_t st) {
  if (n_targets <= 0) return hipSuccess;
  const int nb = (n_targets + kScanBlock - 1) / kScanBlock;
  int32_t* bsum = a.cursor + n_targets + 1;   // nb + 1 scratch words after the cursors
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(nb), dim3(256), 0, st, a, n_targets, bsum);
  hipLaunchKernelGGL(scan_totals_kernel, dim3(1), dim3(256), 0, st, bsum, nb);
  hipLaunchKernelGGL(scan_add_kernel, dim3((n_targets + 255) / 256), dim3(256), 0, st, a, n_targets,
                     (const int32_t*)bsum, nb);
  const int64_t n = (int64_t)a.b * a.R;
  hipLaunchKernelGGL(reverse_scatter_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

// One wave per target: candidates = alive row entries (stored distances) and
// the new vertices pointing at it, the `cap` smallest in (d,id) order, pruned
// against the pre-batch rows of old vertices and the forward rows of new ones.
__device__ void reverse_prune_one(ReverseArgs a, int k, unsigned char* smem);
__global__ __launch_bounds__(64) void reverse_prune_kernel(ReverseArgs a, int n_targets) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int k = blockIdx.x; k < n_targets; k += gridDim.x) {
    reverse_prune_one(a, k, smem);
    __syncthreads();
  }
}
__device__ void reverse_prune_one(ReverseArgs a, int k, unsigned char* smem) {
  const int lane = lane_id();
  const int cap = a.cap;
  WaveCtx w;
  w.ktrack = 0;
  // The merge buffers (next, kept) share the prune table's LDS: the table is
  // built only once the pool is complete, and the pool is then moved back to
  // its own region if the last merge left it in the shared one.
  uint64_t* pool = reinterpret_cast<uint64_t*>(smem + reverse_table_bytes(cap));
  w.pool = pool;
  w.next = reinterpret_cast<uint64_t*>(smem);
  w.kept = w.next + cap;
  w.L = cap;
  for (int i = lane; i < cap; i += kWave) { w.pool[i] = kKeyInf; w.next[i] = kKeyInf; }
  __syncthreads();
  const int32_t t = a.tlist[k];
  const int lo = a.off[k], hi = a.off[k + 1];
  int na = 0;
  bool placed = false;
  uint64_t key = kKeyInf;       // lane r: alive entry r of the row (R <= 64)
  uint64_t ab = 0;              // lanes holding one
  if (a.R <= kWave) {
    // Rows are stored in (d, id) order, so the alive entries fill the empty
    // pool as they stand; a row out of order is merged key by key instead.
    if (lane < a.R) {
      const int32_t u = a.graph[(int64_t)t * a.R + lane];
      const float d = a.edge_d[(int64_t)t * a.R + lane];
      if (u >= 0 && alive_bit(a.alive, u)) key = make_key(d, u);
    }
    ab = ballot(key != kKeyInf);
    na = popc64(ab);
    if (key != kKeyInf) w.pool[lanes_below(ab)] = key;
    __syncthreads();
    const bool bad = lane + 1 < na && key_ord(w.pool[lane]) >= key_ord(w.pool[lane + 1]);
    placed = ballot(bad) == 0;
    __syncthreads();
    if (!placed) {
      if (lane < na) w.pool[lane] = kKeyInf;
      na = 0;
      __syncthreads();
    }
  }
  for (int r0 = 0; !placed && r0 < a.R; r0 += kWave) {
    const int r = r0 + lane;
    uint64_t key = kKeyInf;
    if (r < a.R) {
      const int32_t u = a.graph[(int64_t)t * a.R + r];
      if (u >= 0 && alive_bit(a.alive, u)) key = make_key(a.edge_d[(int64_t)t * a.R + r], u);
    }
    na += popc64(ballot(key != kKeyInf));
    sort_merge(w, key);
  }
  // a list longer than the pool is queued whole for the long-list kernels
  if (a.long_q && na + (hi - lo) > cap) {
    if (lane == 0) {
      const int q = atomicAdd(a.long_n, 1);
      a.long_q[q] = k;
      a.long_len[q] = na + (hi - lo);
    }
    return;
  }
  // With the row in place and at most one wave of incoming keys that all fit,
  // every key's final position is its rank: an alive entry moves up by the
  // incoming keys below it, an incoming key lands after the alive entries and
  // the incoming keys below it.  Equal keys (never produced by one batch) take
  // the merge below, which drops repeats.
  const int c = hi - lo;
  bool merged = false;
  if (placed && c <= kWave && na + c <= cap) {
    const uint64_t q = lane < c ? a.inc[lo + lane] : kKeyInf;
    const bool has_a = key != kKeyInf, has_q = lane < c;
    const uint64_t ko = key_ord(key), qo = key_ord(q);
    const uint32_t q_lo = (uint32_t)q, q_hi = (uint32_t)(q >> 32);
    int up = 0, qpos = 0;
    bool tie = false;
    for (int j = 0; j < c; ++j) {
      const uint64_t qj = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(q_hi, j) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane(q_lo, j);
      const uint64_t qjo = key_ord(qj);
      if (has_a && qjo < ko) ++up;
      const int pa = popc64(ballot(has_a && ko < qjo));
      const int pq = popc64(ballot(has_q && qo < qjo));
      tie = tie || ballot((has_a && ko == qjo) || (has_q && lane != j && qo == qjo)) != 0;
      if (lane == j) qpos = pa + pq;
    }
    if (!tie) {
      if (has_a) pool[lanes_below(ab) + up] = key;
      if (has_q) pool[qpos] = q;
      __syncthreads();
      merged = true;
    }
  }
  for (int c0 = lo; !merged && c0 < hi; c0 += kWave) {
    const int i = c0 + lane;
    uint64_t key = i < hi ? a.inc[i] : kKeyInf;
    sort_merge(w, key);
  }
  if (w.pool != pool) {
    for (int i = lane; i < cap; i += kWave) pool[i] = w.pool[i];
    __syncthreads();
  }
  const int m = merged ? na + c : count_keys(pool, cap);
  PruneLds s = carve_prune_lds(smem, cap);
  RowSource rs{a.graph, a.fwd_ids, a.rows_below ? a.rows_below : a.n0, a.R};
  prune_core(pool, m, rs, a.R, s, a.trow + (int64_t)k * a.R, a.trow_d + (int64_t)k * a.R);
}
hipError_t launch_reverse_prune(const ReverseArgs& a, int n_targets, hipStream_t st) {
  if (n_targets <= 0) return hipSuccess;
  const size_t lds = (size_t)reverse_table_bytes(a.cap) + (size_t)a.cap * 8;
  const int blocks = (int)std::min<int64_t>(n_targets, kMaxBlocks);
  hipLaunchKernelGGL(reverse_prune_kernel, dim3(blocks), dim3(kWave), lds, st, a, n_targets);
  return hipGetLastError();
}

// Raw keys of the queued targets: alive row entries with their stored
// distances, then the incoming keys.  One wave per queued target.
__global__ __launch_bounds__(64) void reverse_gather_kernel(ReverseArgs a, const int32_t* qk,
                                                           LongLists L) {
  const int l = blockIdx.x;
  const int lane = lane_id();
  const int k = qk[l];
  const int32_t t = a.tlist[k];
  uint64_t* out = L.keys + L.off[l];
  int pos = 0;
  for (int r0 = 0; r0 < a.R; r0 += kWave) {
    const int r = r0 + lane;
    const int32_t u = r < a.R ? a.graph[(int64_t)t * a.R + r] : -1;
    const bool ok = u >= 0 && alive_bit(a.alive, u);
    const uint64_t ob = ballot(ok);
    if (ok) out[pos + lanes_below(ob)] = make_key(a.edge_d[(int64_t)t * a.R + r], u);
    pos += popc64(ob);
  }
  const int lo = a.off[k], hi = a.off[k + 1];
  for (int i = lo + lane; i < hi; i += kWave) out[pos + (i - lo)] = a.inc[i];
}
hipError_t launch_reverse_gather(const ReverseArgs& a, const int32_t* qk, const LongLists& L,
                                 hipStream_t st) {
  if (L.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(reverse_gather_kernel, dim3(L.n), dim3(kWave), 0, st, a, qk, L);
  return hipGetLastError();
}

// Commit of a batch: target rows, forward rows of the new ids, alive bits,
// and reset of the per-target counts.
__global__ void commit_targets_kernel(ReverseArgs a, int n_targets, int32_t* graph, float* edge_d) {
  const int64_t n = (int64_t)n_targets * a.R;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(i / a.R), r = (int)(i - (int64_t)k * a.R);
    const int32_t t = a.tlist[k];
    graph[(int64_t)t * a.R + r] = a.trow[i];
    edge_d[(int64_t)t * a.R + r] = a.trow_d[i];
    if (r == 0) a.tcount[t] = 0;
  }
}
__global__ void commit_new_kernel(ReverseArgs a, int32_t* graph, float* edge_d, uint32_t* alive) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)a.b * a.R) return;
  graph[(int64_t)a.n0 * a.R + i] = a.fwd_ids[i];
  edge_d[(int64_t)a.n0 * a.R + i] = a.fwd_d[i];
  if (i % a.R == 0) {
    const int64_t id = a.n0 + i / a.R;
    atomicOr(&alive[id >> 5], 1u << (id & 31));
  }
}
hipError_t launch_commit_batch(const ReverseArgs& a, int n_targets, int32_t* graph, float* edge_d,
                               uint32_t* alive, hipStream_t st) {
  if (n_targets > 0) {
    const int64_t n = (int64_t)n_targets * a.R;
    hipLaunchKernelGGL(commit_targets_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, kMaxBlocks)),
                       dim3(256), 0, st, a, n_targets, graph, edge_d);
  }
  const int64_t n = (int64_t)a.b * a.R;
  if (n > 0)
    hipLaunchKernelGGL(commit_new_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a,
                       graph, edge_d, alive);
  return hipGetLastError();
}

// In-degrees from alive vertices, kept current under updates (used by the
// tiered store's placement).  A row that is rewritten moves one count from
// each entry it drops to each entry it gains; both rows are sets of ids.  One
// 64-lane workgroup per row, both rows staged in LDS (degree <= 128).
__global__ __launch_bounds__(64) void indegree_rows_delta_kernel(const int32_t* __restrict__ graph,
                                                                 const int32_t* __restrict__ list,
                                                                 const int32_t* __restrict__ rows,
                                                                 int n, int R, int32_t* __restrict__ e_in) {
  __shared__ int32_t old_r[128], new_r[128];
  for (int k = blockIdx.x; k < n; k += gridDim.x) {
    const int64_t t = list[k];
    for (int r = threadIdx.x; r < R; r += kWave) {
      old_r[r] = graph[t * R + r];
      new_r[r] = rows[(int64_t)k * R + r];
    }
    __syncthreads();
    for (int r = threadIdx.x; r < R; r += kWave) {
      const int32_t o = old_r[r], w = new_r[r];
      bool o_kept = false, w_had = false;
      for (int j = 0; j < R; ++j) {
        o_kept |= new_r[j] == o;
        w_had |= old_r[j] == w;
      }
      if (o >= 0 && !o_kept) atomicSub(&e_in[o], 1);
      if (w >= 0 && !w_had) atomicAdd(&e_in[w], 1);
    }
    __syncthreads();
  }
}
hipError_t launch_indegree_rows_delta(const int32_t* graph, const int32_t* list, int n,
                                      const int32_t* rows, int R, int32_t* e_in, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (R > 128) return hipErrorInvalidValue;
  hipLaunchKernelGGL(indegree_rows_delta_kernel, dim3((unsigned)std::min<int64_t>(n, kMaxBlocks)),
                     dim3(kWave), 0, st, graph, list, rows, n, R, e_in);
  return hipGetLastError();
}
// Rows of vertices that become alive: one count to each entry.
__global__ void indegree_add_kernel(const int32_t* __restrict__ rows, int64_t n,
                                    int32_t* __restrict__ e_in) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t x = rows[i];
  if (x >= 0) atomicAdd(&e_in[x], 1);
}
hipError_t launch_indegree_add(const int32_t* rows, int64_t n, int32_t* e_in, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(indegree_add_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rows,
                     n, e_in);
  return hipGetLastError();
}

// Bits of the listed ids.
__global__ void mark_list_kernel(const int32_t* list, int n, uint32_t* mask) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicOr(&mask[(uint32_t)list[i] >> 5], 1u << (list[i] & 31));
}
hipError_t launch_mark_list(const int32_t* list, int n, uint32_t* mask, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(mark_list_kernel, dim3((n + 255) / 256), dim3(256), 0, st, list, n, mask);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Deletion (Sec. 5.2).  With in-degrees kept (e_in non-null), a vertex that
// dies takes one count from each entry of its row.
__global__ void mark_deleted_kernel(const int32_t* ids, int64_t n, uint32_t* alive, int32_t* newly,
                                    const int32_t* graph, int R, int32_t* e_in) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t id = ids[i];
  const uint32_t bit = 1u << (id & 31);
  const uint32_t old = atomicAnd(&alive[(uint32_t)id >> 5], ~bit);
  if (old & bit) {
    atomicAdd(newly, 1);
    if (e_in)
      for (int r = 0; r < R; ++r) {
        const int32_t x = graph[(int64_t)id * R + r];
        if (x >= 0) atomicSub(&e_in[x], 1);
      }
  }
}
hipError_t launch_mark_deleted(const int32_t* ids, int64_t n, uint32_t* alive, int32_t* newly,
                               const int32_t* graph, int R, int32_t* e_in, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(mark_deleted_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ids,
                     n, alive, newly, graph, R, e_in);
  return hipGetLastError();
}

// Affected vertices: alive rows with more than half of their valid entries
// deleted (repair) or with any deleted entry (consolidation).  One wave per
// row, grid-stride.
__global__ __launch_bounds__(256) void affected_kernel(RepairArgs a) {
  const int lane = lane_id();
  const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t v = wave; v < a.n_slots; v += nwaves) {
    if (!alive_bit(a.alive, (int32_t)v)) continue;
    int nv = 0, nd = 0;
    for (int r0 = 0; r0 < a.R; r0 += kWave) {
      const int r = r0 + lane;
      const int32_t e = r < a.R ? a.graph[v * a.R + r] : -1;
      const bool valid = e >= 0;
      nv += popc64(ballot(valid));
      nd += popc64(ballot(valid && !alive_bit(a.alive, e)));
    }
    const bool aff = a.consolidate ? nd >= 1 : 2 * nd > nv;
    if (aff && lane == 0) a.list[atomicAdd(a.n_list, 1)] = (int32_t)v;
  }
}
hipError_t launch_affected(const RepairArgs& a, hipStream_t st) {
  if (a.n_slots <= 0) return hipSuccess;
  int64_t blocks = ((int64_t)a.n_slots + 3) / 4;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(affected_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

// Candidates of an affected vertex v: its alive neighbours, then for each
// deleted neighbour p (row order) the first c entries of p's row that are
// alive, not v and not yet candidates.  All distances are evaluated against
// v's own vector.  The `cap` smallest keys are kept; a list shorter than R is
// queued for a search top-up.  A list that offered more than `cap` keys
// (repeats included) is queued as overflowing, with that count; RAW = true
// runs the same walk for the queued lists and writes every offered key to
// the long-list staging area instead.
template <int NC, bool RAW, bool SEG>
__global__ __launch_bounds__(64) void repair_candidates_kernel(RepairArgs a, int first, int count,
                                                               LongLists L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int bi = blockIdx.x;
  if (bi >= count) return;
  const int li = RAW ? a.over_li[bi] : bi;
  const int lane = lane_id();
  const int cap = a.cap;
  const int32_t v = a.list[first + li];
  WaveCtx w;
  w.ktrack = 0;
  w.pool = reinterpret_cast<uint64_t*>(smem);
  w.next = w.pool + (RAW ? 0 : cap);
  w.kept = w.next + (RAW ? 0 : cap);
  w.cid = reinterpret_cast<int32_t*>(w.kept + (RAW ? 0 : kWave));
  w.vis = reinterpret_cast<uint32_t*>(w.cid + kWave);
  w.L = cap;
  uint64_t* out = RAW ? L.keys + L.off[bi] : nullptr;
  int raw = 0;
  const bool exact = a.c < a.R;       // "first c" needs exact membership
  int H = 64;
  if (exact) while (H < 2 * a.R * (1 + a.c)) H <<= 1;
  w.tmask = (uint32_t)H - 1u;
  if (!RAW) for (int i = lane; i < 2 * cap; i += kWave) w.pool[i] = kKeyInf;
  if (exact) for (int i = lane; i < H; i += kWave) w.vis[i] = kEmpty;
  // vectors: the FP32 store in HBM, or the tiered store's host segments (SEG)
  const float* xv = SEG ? a.hsegs.row(v, a.stride) : a.vec32 + (int64_t)v * a.stride;
  auto gather = [&](const QuerySlice<float, NC>& qs, int m) {
    return gather_keys<float, NC, SEG>(qs, a.vec32, a.stride, w.cid, m, a.metric, nullptr, nullptr,
                                       nullptr, a.hsegs);
  };
  QuerySlice<float, NC> q;
  q.load(xv, a.dim, lane % QuerySlice<float, NC>::kLanesPerVec);
  __syncthreads();
  auto take = [&](uint64_t k, int m) {
    if constexpr (RAW) {
      if (lane < m) out[raw + lane] = k;
    } else {
      sort_merge(w, k);
    }
    raw += m;
  };
  const int32_t* rowv = a.graph + (int64_t)v * a.R;
  // alive neighbours
  for (int r0 = 0; r0 < a.R; r0 += kWave) {
    const int r = r0 + lane;
    const int32_t u = r < a.R ? rowv[r] : -1;
    const bool ok = u >= 0 && alive_bit(a.alive, u);
    if (ok && exact) vis_insert_exact(w.vis, w.tmask, u);
    const uint64_t ob = ballot(ok);
    if (ok) w.cid[lanes_below(ob)] = u;
    __syncthreads();
    uint64_t k = gather(q, popc64(ob));
    take(k, popc64(ob));
  }
  // entries of deleted neighbours
  for (int r = 0; r < a.R; ++r) {
    const int32_t p = rowv[r];
    if (p < 0 || alive_bit(a.alive, p)) continue;
    const int32_t* rowp = a.graph + (int64_t)p * a.R;
    int taken = 0;
    for (int e0 = 0; e0 < a.R && (!exact || taken < a.c); e0 += kWave) {
      const int e = e0 + lane;
      const int32_t u = e < a.R ? rowp[e] : -1;
      bool ok = u >= 0 && u != v && alive_bit(a.alive, u);
      if (exact) {
        if (ok) ok = !vis_contains_exact(w.vis, w.tmask, u);
        const uint64_t cb = ballot(ok);
        ok = ok && taken + lanes_below(cb) < a.c;
        __syncthreads();
        if (ok) vis_insert_exact(w.vis, w.tmask, u);
      }
      const uint64_t ob = ballot(ok);
      if (ok) w.cid[lanes_below(ob)] = u;
      taken += popc64(ob);
      __syncthreads();
      if (ob == 0) continue;
      uint64_t k = gather(q, popc64(ob));
      take(k, popc64(ob));
    }
  }
  if constexpr (!RAW) {
    const int m = count_keys(w.pool, cap);
    for (int i = lane; i < cap; i += kWave) a.cand[(int64_t)li * cap + i] = w.pool[i];
    if (lane == 0) {
      a.mcount[li] = m;
      if (raw > cap && a.over_li) {
        const int o = atomicAdd(a.n_over, 1);
        a.over_li[o] = li;
        a.over_len[o] = raw;
      } else if (m < a.R) {
        const int t = atomicAdd(a.n_topup, 1);
        a.topup[t] = li;
        a.topup_v[t] = v;
      }
    }
  }
}
template <bool RAW, bool SEG>
static void launch_repair_nc(const RepairArgs& a, int first, int count, const LongLists& L,
                             size_t lds, hipStream_t st) {
  const int chunks = (int)((a.stride + 127) / 128);
  dim3 g(count), b(kWave);
  switch (chunks <= 1 ? 1 : chunks <= 2 ? 2 : chunks <= 4 ? 4 : 8) {
    case 1: hipLaunchKernelGGL((repair_candidates_kernel<1, RAW, SEG>), g, b, lds, st, a, first, count, L); break;
    case 2: hipLaunchKernelGGL((repair_candidates_kernel<2, RAW, SEG>), g, b, lds, st, a, first, count, L); break;
    case 4: hipLaunchKernelGGL((repair_candidates_kernel<4, RAW, SEG>), g, b, lds, st, a, first, count, L); break;
    default: hipLaunchKernelGGL((repair_candidates_kernel<8, RAW, SEG>), g, b, lds, st, a, first, count, L); break;
  }
}
hipError_t launch_repair_candidates(const RepairArgs& a, int first, int count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  int H = 64;
  if (a.c < a.R) while (H < 2 * a.R * (1 + a.c)) H <<= 1;
  const size_t lds = (size_t)(2 * a.cap + kWave) * 8 + kWave * 4 + (size_t)H * 4;
  const LongLists L{};
  if (a.hsegs.seg) launch_repair_nc<false, true>(a, first, count, L, lds, st);
  else launch_repair_nc<false, false>(a, first, count, L, lds, st);
  return hipGetLastError();
}
hipError_t launch_repair_raw(const RepairArgs& a, int first, const LongLists& L, hipStream_t st) {
  if (L.n <= 0) return hipSuccess;
  int H = 64;
  if (a.c < a.R) while (H < 2 * a.R * (1 + a.c)) H <<= 1;
  const size_t lds = (size_t)kWave * 4 + (size_t)H * 4;
  if (a.hsegs.seg) launch_repair_nc<true, true>(a, first, L.n, L, lds, st);
  else launch_repair_nc<true, false>(a, first, L.n, L, lds, st);
  return hipGetLastError();
}

// Overflowing repair lists after the long-list sort: a list of at most cap
// distinct candidates goes back to its slot of the candidate buffer (and to
// the top-up queue when it has fewer than R); the others stay with the
// long-list kernels and are marked (mcount -1) for the LDS prune to skip.
__global__ __launch_bounds__(64) void repair_back_kernel(RepairArgs a, int first, LongLists L) {
  const int l = blockIdx.x;
  const int lane = lane_id();
  const int li = a.over_li[l];
  const int m = L.m[l];
  if (m > a.cap) {
    // pruned by the long-list kernels; the LDS prune leaves the list alone
    if (lane == 0) a.mcount[li] = -1;
    return;
  }
  const uint64_t* src = L.keys + L.off[l];
  for (int i = lane; i < a.cap; i += kWave) a.cand[(int64_t)li * a.cap + i] = i < m ? src[i] : kKeyInf;
  if (lane == 0) {
    a.mcount[li] = m;
    if (m < a.R) {
      const int t = atomicAdd(a.n_topup, 1);
      a.topup[t] = li;
      a.topup_v[t] = a.list[first + li];
    }
  }
}
hipError_t launch_repair_back(const RepairArgs& a, int first, const LongLists& L, hipStream_t st) {
  if (L.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(repair_back_kernel, dim3(L.n), dim3(kWave), 0, st, a, first, L);
  return hipGetLastError();
}

// Merge the search pool of a topped-up vertex (its own id excluded) into its
// candidate list.
__global__ __launch_bounds__(64) void topup_merge_kernel(RepairArgs a, const uint64_t* pool, int L,
                                                         int ntop) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int ti = blockIdx.x;
  if (ti >= ntop) return;
  const int lane = lane_id();
  const int cap = a.cap;
  const int li = a.topup[ti];
  const int32_t v = a.topup_v[ti];
  WaveCtx w;
  w.ktrack = 0;
  w.pool = reinterpret_cast<uint64_t*>(smem);
  w.next = w.pool + cap;
  w.kept = w.next + cap;
  w.L = cap;
  uint64_t* dst = a.cand + (int64_t)li * cap;
  for (int i = lane; i < cap; i += kWave) { w.pool[i] = dst[i]; w.next[i] = kKeyInf; }
  __syncthreads();
  for (int c0 = 0; c0 < L; c0 += kWave) {
    const int i = c0 + lane;
    uint64_t k = i < L ? pool[(int64_t)ti * L + i] : kKeyInf;
    if (key_id(k) == v) k = kKeyInf;
    sort_merge(w, k);
  }
  const int m = count_keys(w.pool, cap);
  for (int i = lane; i < cap; i += kWave) dst[i] = w.pool[i];
  if (lane == 0) a.mcount[li] = m;
}
hipError_t launch_topup_merge(const RepairArgs& a, const uint64_t* pool, int L, int first,
                              int ntop, hipStream_t st) {
  (void)first;
  if (ntop <= 0) return hipSuccess;
  const size_t lds = (size_t)(2 * a.cap + kWave) * 8;
  hipLaunchKernelGGL(topup_merge_kernel, dim3(ntop), dim3(kWave), lds, st, a, pool, L, ntop);
  return hipGetLastError();
}

__global__ void commit_rows_kernel(const int32_t* list, int n, const int32_t* rows,
                                   const float* rows_d, int R, int32_t* graph, float* edge_d) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < (int64_t)n * R;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(i / R), r = (int)(i - (int64_t)k * R);
    const int64_t v = list[k];
    graph[v * R + r] = rows[i];
    edge_d[v * R + r] = rows_d[i];
  }
}
hipError_t launch_commit_rows(const int32_t* list, int n, const int32_t* rows, const float* rows_d,
                              int R, int32_t* graph, float* edge_d, hipStream_t st) {
  const int64_t t = (int64_t)n * R;
  if (t <= 0) return hipSuccess;
  hipLaunchKernelGGL(commit_rows_kernel, dim3((unsigned)std::min<int64_t>((t + 255) / 256, kMaxBlocks)),
                     dim3(256), 0, st, list, n, rows, rows_d, R, graph, edge_d);
  return hipGetLastError();
}

}  // namespace svf
