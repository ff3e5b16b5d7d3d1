// Entry/stop predictor kernels: BF16 MFMA GEMM with fused epilogues, loss and
// gradient, Adam, the gating decision, and k-means for the entry clusters.
#include "mlp.hpp"

#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"

namespace svf {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// C (M x N) = A (M x K) * B (K x N) on BF16 operands with FP32 accumulation.
// A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn] (strides in elements),
// so transposed operands need no copies.  A 256-thread workgroup owns a 64x64
// tile; each wave a 32x32 block computed with v_mfma_f32_32x32x8_bf16 (lane l
// feeds row/column l % 32 and k-quad l / 32; the 16 results of lane l are
// rows 8*(r/4) + 4*(l/32) + r%4, column l % 32).
// Epilogue: + bias[n], then ReLU (relu) or zeroing where mask(m,n) <= 0, then
// FP32 and/or BF16 stores with leading dimension ldc.
struct GemmArgs {
  const uint16_t* A; int64_t sam, sak;
  const uint16_t* B; int64_t sbk, sbn;
  int M, N, K;
  const float* bias;
  int relu;
  const float* mask; int64_t ldm;
  float* C32; uint16_t* C16; int64_t ldc;
};

__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 64 + (wv >> 1) * 32;
  const int n0 = blockIdx.x * 64 + (wv & 1) * 32;
  const int rc = lane & 31, kq = (lane >> 5) * 4;
  const int row = m0 + rc, col = n0 + rc;
  v16f acc = {};
  for (int k0 = 0; k0 < g.K; k0 += 8) {
    v4s a, b;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int kk = k0 + kq + i;
      a[i] = (row < g.M && kk < g.K) ? (short)g.A[row * g.sam + kk * g.sak] : (short)0;
      b[i] = (col < g.N && kk < g.K) ? (short)g.B[kk * g.sbk + col * g.sbn] : (short)0;
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = m0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    const int n = n0 + rc;
    if (m >= g.M || n >= g.N) continue;
    float v = acc[r];
    if (g.bias) v += g.bias[n];
    if (g.relu) v = v > 0.f ? v : 0.f;
    if (g.mask && !(g.mask[m * g.ldm + n] > 0.f)) v = 0.f;
    if (g.C32) g.C32[m * g.ldc + n] = v;
    if (g.C16) g.C16[m * g.ldc + n] = f32_to_bf16_rne(v);
  }
}

static hipError_t gemm(const GemmArgs& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  dim3 grid((g.N + 63) / 64, (g.M + 63) / 64);
  hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

__global__ void to_bf16_kernel(const float* x, int64_t rows, int cols, int64_t ldx, uint16_t* y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const int64_t r = i / cols, c = i - r * cols;
  y[i] = f32_to_bf16_rne(x[r * ldx + c]);
}

// Column sums of an n x cols FP32 matrix: a block of 1024 threads covers 64
// columns, its 16 waves take every 16th row, and the 16 partial sums are
// added in wave order (the same order on every run).
__global__ __launch_bounds__(1024) void colsum_kernel(const float* x, int64_t rows, int cols,
                                                      float* out) {
  __shared__ float part[16][64];
  const int cl = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + cl;
  float s = 0.f;
  if (c < cols)
    for (int64_t r = wv; r < rows; r += 16) s += x[r * cols + c];
  part[wv][cl] = s;
  __syncthreads();
  if (wv == 0 && c < cols) {
    float t = 0.f;
    for (int k = 0; k < 16; ++k) t += part[k][cl];
    out[c] = t;
  }
}

__device__ __forceinline__ float wave_max(float v) {
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// One wave per sample: softmax cross-entropy on the nc logits and lambda *
// Huber on the stop output; gradients scaled by 1/n (the batch mean).
__global__ __launch_bounds__(256) void loss_grad_kernel(const float* z, const int32_t* label,
                                                        const float* log_stop, int64_t n, int nc,
                                                        float lambda, float delta, float* dzf,
                                                        uint16_t* dzb, float* loss) {
  const int64_t i = blockIdx.x * (int64_t)(blockDim.x / 64) + threadIdx.x / 64;
  if (i >= n) return;
  const int lane = threadIdx.x & 63;
  const int no = nc + 1;
  const float* zi = z + i * no;
  float mx = -__builtin_inff();
  for (int j = lane; j < nc; j += 64) mx = fmaxf(mx, zi[j]);
  mx = wave_max(mx);
  float se = 0.f;
  for (int j = lane; j < nc; j += 64) se += __expf(zi[j] - mx);
  se = wave_sum(se);
  const int lab = label[i];
  const float inv = 1.0f / (float)n;
  for (int j = lane; j < nc; j += 64) {
    const float gj = (__expf(zi[j] - mx) / se - (j == lab ? 1.f : 0.f)) * inv;
    dzf[i * no + j] = gj;
    dzb[i * no + j] = f32_to_bf16_rne(gj);
  }
  if (lane == 0) {
    float l = logf(se) + mx - zi[lab];
    const float r = zi[nc] - log_stop[i];
    const float ar = fabsf(r);
    l += lambda * (ar <= delta ? 0.5f * r * r : delta * (ar - 0.5f * delta));
    const float gs = lambda * (ar <= delta ? r : (r > 0.f ? delta : -delta)) * inv;
    dzf[i * no + nc] = gs;
    dzb[i * no + nc] = f32_to_bf16_rne(gs);
    atomicAdd(loss, l * inv);
  }
}

__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void round_params_kernel(float* p, uint16_t* wb, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint16_t b = f32_to_bf16_rne(p[i]);
  wb[i] = b;
}

// Gating of the learned form: the first largest cluster logit, its softmax
// probability p = 1 / sum_j exp(z_j - z_max), and with p >= conf the cluster
// and an expansion cap max(min_iters, ceil(stop_scale * exp(min(z_stop, 20))))
// held at or below 2^30; otherwise plain search (cluster -1, no cap), counted
// in *n_fallback when given.
__global__ void decide_kernel(const float* z, int64_t n, int nc, float conf, float stop_scale,
                              int min_iters, int32_t* q_entry, int32_t* q_max,
                              unsigned long long* n_fallback) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* zi = z + i * (nc + 1);
  int best = 0;
  float mx = zi[0];
  for (int j = 1; j < nc; ++j)
    if (zi[j] > mx) { mx = zi[j]; best = j; }
  float se = 0.f;
  for (int j = 0; j < nc; ++j) se += __expf(zi[j] - mx);
  const float p = 1.0f / se;                  // softmax of the argmax
  if (p >= conf) {
    q_entry[i] = best;
    const float cap = fminf(ceilf(stop_scale * __expf(fminf(zi[nc], 20.f))), 1073741824.f);
    const int c = (int)cap;
    q_max[i] = c < min_iters ? min_iters : c;
  } else {
    q_entry[i] = -1;
    q_max[i] = 0;
    if (n_fallback) atomicAdd(n_fallback, 1ull);
  }
}

hipError_t launch_model_decide(const float* z, int64_t n, int nc, float conf, float stop_scale,
                               int min_iters, int32_t* q_entry, int32_t* q_max_iters,
                               unsigned long long* n_fallback, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(decide_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, z, n, nc,
                     conf, stop_scale, min_iters, q_entry, q_max_iters, n_fallback);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k-means.  Assignment: one thread per row, centroids staged in LDS.
__global__ __launch_bounds__(256) void kmeans_assign_kernel(const float* x, int64_t n,
                                                            int64_t stride, int dim,
                                                            const float* cent, int nc,
                                                            const int32_t* ids, int id_step,
                                                            int32_t* assign) {
  extern __shared__ float cs[];
  for (int i = threadIdx.x; i < nc * dim; i += blockDim.x) cs[i] = cent[i];
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t rowi = i;
  if (ids) {
    rowi = ids[i * id_step];
    if (rowi < 0) { assign[i] = -1; return; }
  }
  const float* xr = x + rowi * stride;
  int best = 0;
  float bd = 3.4e38f;
  for (int c = 0; c < nc; ++c) {
    float s = 0.f;
    for (int t = 0; t < dim; ++t) { const float d = xr[t] - cs[c * dim + t]; s = fmaf(d, d, s); }
    if (s < bd) { bd = s; best = c; }
  }
  assign[i] = best;
}

__global__ void kmeans_accum_kernel(const float* x, int64_t n, int64_t stride, int dim,
                                    const int32_t* assign, float* sums, float* counts) {
  const int64_t i = blockIdx.x;
  if (i >= n) return;
  const int c = assign[i];
  for (int t = threadIdx.x; t < dim; t += blockDim.x) atomicAdd(&sums[c * dim + t], x[i * stride + t]);
  if (threadIdx.x == 0) atomicAdd(&counts[c], 1.f);
}

__global__ void kmeans_update_kernel(float* cent, const float* sums, const float* counts, int nc,
                                     int dim) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc * dim) return;
  const float cnt = counts[i / dim];
  if (cnt > 0.f) cent[i] = sums[i] / cnt;
}

hipError_t assign_rows(const float* x, int64_t stride, int dim, const int32_t* ids, int64_t n,
                       int id_step, const float* centroids, int nc, int32_t* assign,
                       hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const size_t lds = (size_t)nc * dim * 4;
  hipLaunchKernelGGL(kmeans_assign_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), lds, st, x,
                     n, stride, dim, centroids, nc, ids, id_step, assign);
  return hipGetLastError();
}

hipError_t kmeans(const float* x, int64_t n, int64_t stride, int dim, int nc, int iters,
                  float* centroids, int32_t* assign, hipStream_t st) {
  float* sums = nullptr;
  hipError_t e = hipMalloc(&sums, (size_t)(nc * dim + nc) * 4);
  if (e != hipSuccess) return e;
  float* counts = sums + nc * dim;
  for (int it = 0; it < iters && e == hipSuccess; ++it) {
    if ((e = assign_rows(x, stride, dim, nullptr, n, 1, centroids, nc, assign, st)) != hipSuccess) break;
    if ((e = launch_fill_u32(sums, nc * dim + nc, 0u, st)) != hipSuccess) break;
    hipLaunchKernelGGL(kmeans_accum_kernel, dim3((unsigned)n), dim3(64), 0, st, x, n, stride, dim,
                       assign, sums, counts);
    hipLaunchKernelGGL(kmeans_update_kernel, dim3((nc * dim + 255) / 256), dim3(256), 0, st,
                       centroids, sums, counts, nc, dim);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = assign_rows(x, stride, dim, nullptr, n, 1, centroids, nc, assign, st);
  hipError_t e2 = hipStreamSynchronize(st);
  (void)hipFree(sums);
  return e != hipSuccess ? e : e2;
}

// Entry lists spread over each cluster: one wave per cluster walks the
// clustered sample (row i of the sample is stored vector i * step) in order,
// counts the cluster's alive members m, and keeps the members of rank
// floor(j * m / ecap), j = 0..ecap-1 (all of them, -1 padded, when m < ecap).
// Sample order is id order, and ids follow no cluster, so the kept members
// are spread over every part of the cluster in proportion to its size.
__global__ __launch_bounds__(64) void spread_entries_kernel(const int32_t* __restrict__ assign,
                                                           int64_t ns, int64_t step,
                                                           const uint32_t* __restrict__ alive,
                                                           int ecap, int32_t* __restrict__ lists) {
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  int32_t* out = lists + (int64_t)c * ecap;
  int64_t m = 0;
  for (int64_t i0 = 0; i0 < ns; i0 += 64) {
    const int64_t i = i0 + lane;
    const bool mem = i < ns && assign[i] == c && alive_bit(alive, (int32_t)(i * step));
    m += __popcll(__ballot(mem));
  }
  for (int j = lane; j < ecap; j += 64) out[j] = -1;
  __syncthreads();
  int64_t r0 = 0;
  for (int64_t i0 = 0; i0 < ns; i0 += 64) {
    const int64_t i = i0 + lane;
    const bool mem = i < ns && assign[i] == c && alive_bit(alive, (int32_t)(i * step));
    const uint64_t b = __ballot(mem);
    if (mem) {
      const int64_t r = r0 + __popcll(b & ((1ull << lane) - 1ull));
      if (m <= ecap) {
        out[r] = (int32_t)(i * step);
      } else {
        // the j with floor(j * m / ecap) == r, if any
        const int64_t j = (r * ecap + m - 1) / m;
        if (j < ecap && (j * m) / ecap == r) out[j] = (int32_t)(i * step);
      }
    }
    r0 += __popcll(b);
  }
}

hipError_t launch_spread_entries(const int32_t* assign, int64_t ns, int64_t step,
                                 const uint32_t* alive, int nc, int ecap, int32_t* lists,
                                 hipStream_t st) {
  if (nc <= 0) return hipSuccess;
  hipLaunchKernelGGL(spread_entries_kernel, dim3(nc), dim3(64), 0, st, assign, ns, step, alive, ecap,
                     lists);
  return hipGetLastError();
}

__global__ void log_steps_kernel(const int32_t* s, int64_t n, float* out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = logf((float)(s[i] > 1 ? s[i] : 1));
}
hipError_t launch_log_steps(const int32_t* steps, int64_t n, float* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(log_steps_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, steps,
                     n, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Host side.
#define MCK(x)                              \
  do {                                      \
    hipError_t e_ = (x);                    \
    if (e_ != hipSuccess) return e_;        \
  } while (0)

static inline unsigned blocks(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

Mlp::Mlp(int din, int h, int nc, uint64_t seed) : d_{din, h, nc}, seed_(seed) {}

Mlp::~Mlp() {
  for (void* p : {(void*)p_, (void*)wb_, (void*)m_, (void*)v_, (void*)g_, (void*)loss_, (void*)xb_,
                  (void*)h1f_, (void*)h1b_, (void*)h2f_, (void*)h2b_, (void*)zf_, (void*)dzf_,
                  (void*)dzb_, (void*)dh2f_, (void*)dh2b_, (void*)dh1f_, (void*)dh1b_})
    if (p) (void)hipFree(p);
}

// He-normal weights from a SplitMix64 stream with Box-Muller, zero biases.
hipError_t Mlp::init_device(hipStream_t st) {
  const int64_t n = d_.total();
  MCK(hipMalloc(&p_, n * 4));
  MCK(hipMalloc(&wb_, n * 2));
  MCK(hipMalloc(&m_, n * 4));
  MCK(hipMalloc(&v_, n * 4));
  MCK(hipMalloc(&g_, n * 4));
  MCK(hipMalloc(&loss_, 16));
  std::vector<float> h(n, 0.f);
  uint64_t s = seed_;
  auto next = [&]() {
    s += 0x9E3779B97F4A7C15ull;
    uint64_t z = s;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return ((z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  };
  auto fill = [&](int64_t off, int64_t cnt, int fan_in) {
    const double sd = std::sqrt(2.0 / fan_in);
    for (int64_t i = 0; i < cnt; ++i) {
      const double u1 = next(), u2 = next();
      h[off + i] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
    }
  };
  fill(d_.o_w1(), (int64_t)d_.din * d_.h, d_.din);
  fill(d_.o_w2(), (int64_t)d_.h * d_.h, d_.h);
  fill(d_.o_w3(), (int64_t)d_.h * d_.no(), d_.h);
  MCK(set_params(h.data(), st));
  return hipSuccess;
}

hipError_t Mlp::refresh_bf16(hipStream_t st) {
  const int64_t n = d_.total();
  hipLaunchKernelGGL(round_params_kernel, dim3(blocks(n)), dim3(256), 0, st, p_, wb_, n);
  return hipGetLastError();
}

hipError_t Mlp::set_params(const float* host, hipStream_t st) {
  const int64_t n = d_.total();
  std::vector<float> r(host, host + n);
  // weights live on the BF16 grid (biases stay FP32)
  auto rnd = [](float x) {
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    float y;
    std::memcpy(&y, &u, 4);
    return y;
  };
  for (int64_t i = d_.o_w1(); i < d_.o_b1(); ++i) r[i] = rnd(r[i]);
  for (int64_t i = d_.o_w2(); i < d_.o_b2(); ++i) r[i] = rnd(r[i]);
  for (int64_t i = d_.o_w3(); i < d_.o_b3(); ++i) r[i] = rnd(r[i]);
  MCK(hipMemcpyAsync(p_, r.data(), n * 4, hipMemcpyHostToDevice, st));
  MCK(launch_fill_u32(m_, n, 0u, st));
  MCK(launch_fill_u32(v_, n, 0u, st));
  MCK(refresh_bf16(st));
  MCK(hipStreamSynchronize(st));
  step_ = 0;
  return hipSuccess;
}

hipError_t Mlp::get_params(float* host, hipStream_t st) {
  MCK(hipMemcpyAsync(host, p_, d_.total() * 4, hipMemcpyDeviceToHost, st));
  return hipStreamSynchronize(st);
}

hipError_t Mlp::ensure_batch(int64_t n) {
  if (n <= cap_) return hipSuccess;
  for (void* p : {(void*)xb_, (void*)h1f_, (void*)h1b_, (void*)h2f_, (void*)h2b_, (void*)zf_,
                  (void*)dzf_, (void*)dzb_, (void*)dh2f_, (void*)dh2b_, (void*)dh1f_, (void*)dh1b_})
    if (p) (void)hipFree(p);
  const int64_t c = n;
  const int h = d_.h, no = d_.no();
  MCK(hipMalloc(&xb_, c * d_.din * 2));
  MCK(hipMalloc(&h1f_, c * h * 4));
  MCK(hipMalloc(&h1b_, c * h * 2));
  MCK(hipMalloc(&h2f_, c * h * 4));
  MCK(hipMalloc(&h2b_, c * h * 2));
  MCK(hipMalloc(&zf_, c * no * 4));
  MCK(hipMalloc(&dzf_, c * no * 4));
  MCK(hipMalloc(&dzb_, c * no * 2));
  MCK(hipMalloc(&dh2f_, c * h * 4));
  MCK(hipMalloc(&dh2b_, c * h * 2));
  MCK(hipMalloc(&dh1f_, c * h * 4));
  MCK(hipMalloc(&dh1b_, c * h * 2));
  cap_ = c;
  return hipSuccess;
}

hipError_t Mlp::run_forward(const float* d_x, int64_t n, hipStream_t st) {
  const int din = d_.din, h = d_.h, no = d_.no();
  hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(n * din)), dim3(256), 0, st, d_x, n, din,
                     (int64_t)din, xb_);
  GemmArgs g{};
  g.A = xb_; g.sam = din; g.sak = 1;
  g.B = wb_ + d_.o_w1(); g.sbk = h; g.sbn = 1;
  g.M = (int)n; g.N = h; g.K = din;
  g.bias = p_ + d_.o_b1(); g.relu = 1;
  g.C32 = h1f_; g.C16 = h1b_; g.ldc = h;
  MCK(gemm(g, st));
  g.A = h1b_; g.sam = h;
  g.B = wb_ + d_.o_w2(); g.sbk = h;
  g.K = h; g.bias = p_ + d_.o_b2();
  g.C32 = h2f_; g.C16 = h2b_;
  MCK(gemm(g, st));
  g.A = h2b_;
  g.B = wb_ + d_.o_w3(); g.sbk = no;
  g.N = no; g.bias = p_ + d_.o_b3(); g.relu = 0;
  g.C32 = zf_; g.C16 = nullptr; g.ldc = no;
  MCK(gemm(g, st));
  return hipSuccess;
}

hipError_t Mlp::run_backward(const int32_t* d_label, const float* d_log_stop, int64_t n,
                             float lambda, float delta, float* d_grad, hipStream_t st) {
  const int din = d_.din, h = d_.h, no = d_.no();
  hipLaunchKernelGGL(loss_grad_kernel, dim3(blocks(n, 4)), dim3(256), 0, st, zf_, d_label, d_log_stop,
                     n, d_.nc, lambda, delta, dzf_, dzb_, loss_);
  GemmArgs g{};
  // dW3 = H2^T dZ  (h x no), db3 = colsum dZ
  g.A = h2b_; g.sam = 1; g.sak = h;
  g.B = dzb_; g.sbk = no; g.sbn = 1;
  g.M = h; g.N = no; g.K = (int)n;
  g.C32 = d_grad + d_.o_w3(); g.ldc = no;
  MCK(gemm(g, st));
  hipLaunchKernelGGL(colsum_kernel, dim3(blocks(no, 64)), dim3(1024), 0, st, dzf_, n, no,
                     d_grad + d_.o_b3());
  // dH2 = (dZ W3^T) masked by H2 > 0
  g = GemmArgs{};
  g.A = dzb_; g.sam = no; g.sak = 1;
  g.B = wb_ + d_.o_w3(); g.sbk = 1; g.sbn = no;
  g.M = (int)n; g.N = h; g.K = no;
  g.mask = h2f_; g.ldm = h;
  g.C32 = dh2f_; g.C16 = dh2b_; g.ldc = h;
  MCK(gemm(g, st));
  // dW2 = H1^T dH2, db2
  g = GemmArgs{};
  g.A = h1b_; g.sam = 1; g.sak = h;
  g.B = dh2b_; g.sbk = h; g.sbn = 1;
  g.M = h; g.N = h; g.K = (int)n;
  g.C32 = d_grad + d_.o_w2(); g.ldc = h;
  MCK(gemm(g, st));
  hipLaunchKernelGGL(colsum_kernel, dim3(blocks(h, 64)), dim3(1024), 0, st, dh2f_, n, h,
                     d_grad + d_.o_b2());
  // dH1 = (dH2 W2^T) masked by H1 > 0
  g = GemmArgs{};
  g.A = dh2b_; g.sam = h; g.sak = 1;
  g.B = wb_ + d_.o_w2(); g.sbk = 1; g.sbn = h;
  g.M = (int)n; g.N = h; g.K = h;
  g.mask = h1f_; g.ldm = h;
  g.C32 = dh1f_; g.C16 = dh1b_; g.ldc = h;
  MCK(gemm(g, st));
  // dW1 = X^T dH1, db1
  g = GemmArgs{};
  g.A = xb_; g.sam = 1; g.sak = din;
  g.B = dh1b_; g.sbk = h; g.sbn = 1;
  g.M = din; g.N = h; g.K = (int)n;
  g.C32 = d_grad + d_.o_w1(); g.ldc = h;
  MCK(gemm(g, st));
  hipLaunchKernelGGL(colsum_kernel, dim3(blocks(h, 64)), dim3(1024), 0, st, dh1f_, n, h,
                     d_grad + d_.o_b1());
  return hipGetLastError();
}

hipError_t Mlp::forward(const float* d_x, int64_t n, float* d_out, hipStream_t st) {
  for (int64_t s = 0; s < n; s += 65536) {
    const int64_t b = n - s < 65536 ? n - s : 65536;
    MCK(ensure_batch(b));
    MCK(run_forward(d_x + s * d_.din, b, st));
    MCK(hipMemcpyAsync(d_out + s * d_.no(), zf_, b * d_.no() * 4, hipMemcpyDeviceToDevice, st));
  }
  return hipSuccess;
}

hipError_t Mlp::loss_grad(const float* d_x, const int32_t* d_label, const float* d_log_stop,
                          int64_t n, float lambda, float delta, float* d_grad, float* h_loss,
                          hipStream_t st) {
  MCK(ensure_batch(n));
  MCK(launch_fill_u32(loss_, 1, 0u, st));
  MCK(run_forward(d_x, n, st));
  MCK(run_backward(d_label, d_log_stop, n, lambda, delta, d_grad, st));
  if (h_loss) {
    MCK(hipMemcpyAsync(h_loss, loss_, 4, hipMemcpyDeviceToHost, st));
    MCK(hipStreamSynchronize(st));
  }
  return hipSuccess;
}

hipError_t Mlp::train(const float* d_x, const int32_t* d_label, const float* d_log_stop, int64_t n,
                      int epochs, int batch, float lr, float lambda, float delta,
                      float* h_last_loss, hipStream_t st) {
  const int64_t np = d_.total();
  const float b1 = 0.9f, b2 = 0.999f;
  MCK(ensure_batch(batch));
  for (int ep = 0; ep < epochs; ++ep) {
    MCK(launch_fill_u32(loss_, 1, 0u, st));
    int nb = 0;
    for (int64_t s = 0; s + batch <= n; s += batch, ++nb) {
      MCK(run_forward(d_x + s * d_.din, batch, st));
      MCK(run_backward(d_label + s, d_log_stop + s, batch, lambda, delta, g_, st));
      ++step_;
      const float c1 = 1.f - std::pow(b1, (float)step_), c2 = 1.f - std::pow(b2, (float)step_);
      hipLaunchKernelGGL(adam_kernel, dim3(blocks(np)), dim3(256), 0, st, p_, g_, m_, v_, np, lr,
                         b1, b2, 1e-8f, c1, c2);
      MCK(refresh_bf16(st));
    }
    if (h_last_loss && ep == epochs - 1) {
      float l = 0.f;
      MCK(hipMemcpyAsync(&l, loss_, 4, hipMemcpyDeviceToHost, st));
      MCK(hipStreamSynchronize(st));
      *h_last_loss = nb > 0 ? l / nb : 0.f;
    }
  }
  return hipStreamSynchronize(st);
}

}  // namespace svf
