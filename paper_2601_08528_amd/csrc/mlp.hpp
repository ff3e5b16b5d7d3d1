// Entry/stop predictor (host side): a din -> H -> H -> (NC + 1) perceptron
// with ReLU, BF16 weights and activations, FP32 accumulation on MFMA, FP32
// master weights and Adam.  Outputs 0..NC-1 are logits of the cluster whose
// entry list should start a query's search; output NC predicts the log of the
// expansion count after which the query's top-k stops changing.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace svf {

struct MlpDims {
  int din, h, nc;
  int no() const { return nc + 1; }
  // offsets of W1 b1 W2 b2 W3 b3 in the flat FP32 parameter vector
  int64_t o_w1() const { return 0; }
  int64_t o_b1() const { return (int64_t)din * h; }
  int64_t o_w2() const { return o_b1() + h; }
  int64_t o_b2() const { return o_w2() + (int64_t)h * h; }
  int64_t o_w3() const { return o_b2() + h; }
  int64_t o_b3() const { return o_w3() + (int64_t)h * no(); }
  int64_t total() const { return o_b3() + no(); }
};

class Mlp {
 public:
  Mlp(int din, int h, int nc, uint64_t seed);
  ~Mlp();
  hipError_t init_device(hipStream_t st);
  const MlpDims& dims() const { return d_; }
  // host FP32 parameters in the flat order; weights are kept on the BF16 grid
  hipError_t set_params(const float* host, hipStream_t st);
  hipError_t get_params(float* host, hipStream_t st);
  // z = forward(x) for n rows of FP32 input (device), output n x (nc+1) FP32 (device)
  hipError_t forward(const float* d_x, int64_t n, float* d_out, hipStream_t st);
  // mean loss and its gradient (flat FP32, device) for one batch
  hipError_t loss_grad(const float* d_x, const int32_t* d_label, const float* d_log_stop, int64_t n,
                       float lambda, float delta, float* d_grad, float* h_loss, hipStream_t st);
  // Adam over `epochs` passes of mini-batches (device data, n rows)
  hipError_t train(const float* d_x, const int32_t* d_label, const float* d_log_stop, int64_t n,
                   int epochs, int batch, float lr, float lambda, float delta, float* h_last_loss,
                   hipStream_t st);
  int64_t steps() const { return step_; }

 private:
  hipError_t ensure_batch(int64_t n);
  hipError_t run_forward(const float* d_x, int64_t n, hipStream_t st);
  hipError_t run_backward(const int32_t* d_label, const float* d_log_stop, int64_t n, float lambda,
                          float delta, float* d_grad, hipStream_t st);
  hipError_t refresh_bf16(hipStream_t st);

  MlpDims d_;
  uint64_t seed_;
  int64_t step_ = 0;
  float* p_ = nullptr;        // FP32 master parameters
  uint16_t* wb_ = nullptr;    // BF16 copy of the parameters (weights used by GEMMs)
  float* m_ = nullptr;        // Adam moments
  float* v_ = nullptr;
  float* g_ = nullptr;        // gradient scratch
  float* loss_ = nullptr;     // device loss accumulator
  int64_t cap_ = 0;
  uint16_t* xb_ = nullptr;    // batch input BF16
  float* h1f_ = nullptr; uint16_t* h1b_ = nullptr;
  float* h2f_ = nullptr; uint16_t* h2b_ = nullptr;
  float* zf_ = nullptr;
  float* dzf_ = nullptr; uint16_t* dzb_ = nullptr;
  float* dh2f_ = nullptr; uint16_t* dh2b_ = nullptr;
  float* dh1f_ = nullptr; uint16_t* dh1b_ = nullptr;
};

// Gate of the learned form: per query the argmax cluster and its softmax
// probability; queries at or above conf get that cluster's entry list and a
// cap of ceil(stop_scale * exp(z_stop)) expansions (at least min_iters),
// others keep random entries and no cap (plain search).
hipError_t launch_model_decide(const float* z, int64_t n, int nc, float conf, float stop_scale,
                               int min_iters, int32_t* q_entry, int32_t* q_max_iters,
                               unsigned long long* n_fallback, hipStream_t st);

// Lloyd k-means of n rows (stride `stride`, first dim used) into nc centroids
// (device, nc x dim), `iters` iterations, initial centroids given.
hipError_t kmeans(const float* x, int64_t n, int64_t stride, int dim, int nc, int iters,
                  float* centroids, int32_t* assign, hipStream_t st);
// assign[i] = nearest centroid of row ids[i] of x (stride), ids -1 -> -1
hipError_t assign_rows(const float* x, int64_t stride, int dim, const int32_t* ids, int64_t n,
                       int id_step, const float* centroids, int nc, int32_t* assign, hipStream_t st);
// Per cluster, ecap entry ids spread over its alive members in the clustered
// sample (sample row i = stored vector i * step), -1 padded.
hipError_t launch_spread_entries(const int32_t* assign, int64_t ns, int64_t step,
                                 const uint32_t* alive, int nc, int ecap, int32_t* lists,
                                 hipStream_t st);
// log(max(1, steps)) as FP32
hipError_t launch_log_steps(const int32_t* steps, int64_t n, float* out, hipStream_t st);

}  // namespace svf
