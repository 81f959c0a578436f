// Surrogate network of the transmutation energy (10 -> 64 -> 64 -> 1, SiLU,
// BF16 operands on the 16x16x32 MFMA, FP32 accumulation): inference,
// normalization fitting, and training with hand-written forward/backward
// kernels and Adam on FP32 master weights.
//
// Parameter order of the flat vectors (4929 values):
//   w1[64][10], b1[64], w2[64][64], b2[64], w3[64], b3.
#include <cmath>
#include <vector>

#include "mlp_device.hpp"

namespace vc {

constexpr int OFF_W1 = 0, OFF_B1 = 640, OFF_W2 = 704, OFF_B2 = 4800, OFF_W3 = 4864, OFF_B3 = 4928;

}  // namespace vc

struct vcsgc_mlp {
  hipStream_t stream = nullptr;
  int device = 0;
  float *p = nullptr;     // FP32 master parameters [4929]
  float *g = nullptr;     // gradient [4929]
  float *m1 = nullptr, *m2 = nullptr;  // Adam moments
  __bf16 *w1b = nullptr;  // [64][32]
  __bf16 *w2b = nullptr;  // [64][64]
  float *w3r = nullptr;   // [64] bf16-rounded w3
  float mu[10], sd[10];
  float out_mu = 0.f, out_sd = 1.f;
  int64_t adam_t = 0;
  // training scratch for batch size cap
  int64_t cap = 0;
  float *Z = nullptr, *T = nullptr, *A1 = nullptr, *H1 = nullptr, *A2 = nullptr, *H2 = nullptr;
  float *Y = nullptr, *dY = nullptr, *dA2 = nullptr, *dH1 = nullptr, *dA1 = nullptr;
  double *red = nullptr;  // loss / statistics partials
  std::string err;
};

namespace vc {

MlpDev mlp_dev(const vcsgc_mlp *m) {
  MlpDev d;
  d.w1 = m->w1b;
  d.w2 = m->w2b;
  d.b1 = m->p + OFF_B1;
  d.b2 = m->p + OFF_B2;
  d.w3 = m->w3r;
  d.b3 = m->p + OFF_B3;
  for (int k = 0; k < MLP_IN; ++k) {
    d.mu[k] = m->mu[k];
    d.sd[k] = m->sd[k];
  }
  d.out_mu = m->out_mu;
  d.out_sd = m->out_sd;
  return d;
}

// bf16 copies of the weights for the MFMA operands
__global__ void k_mlp_refresh(const float *__restrict__ p, __bf16 *w1b, __bf16 *w2b, float *w3r) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < MLP_H * MLP_KP) {
    const int n = t / MLP_KP, k = t % MLP_KP;
    w1b[t] = to_bf16(k < MLP_IN ? p[OFF_W1 + n * MLP_IN + k] : 0.0f);
  }
  if (t < MLP_H * MLP_H) w2b[t] = to_bf16(p[OFF_W2 + t]);
  if (t < MLP_H) w3r[t] = bf16_round(p[OFF_W3 + t]);
}

hipError_t mlp_refresh(vcsgc_mlp *m) {
  k_mlp_refresh<<<16, 256, 0, m->stream>>>(m->p, m->w1b, m->w2b, m->w3r);
  return hipGetLastError();
}

// Inference on n raw descriptors (FP64, [n][10]); 16 samples per block.
__global__ void __launch_bounds__(BLOCK) k_mlp_infer(MlpDev md, int64_t n,
                                                     const double *__restrict__ desc, double *dE) {
  __shared__ __bf16 zs[16 * MLP_KP];
  __shared__ __bf16 h1[16 * MLP_H], h2[16 * MLP_H];
  __shared__ float yv[16];
  const int64_t base = (int64_t)blockIdx.x * 16;
  for (int e = threadIdx.x; e < 16 * MLP_KP; e += BLOCK) {
    const int r = e / MLP_KP, k = e % MLP_KP;
    const int64_t b = base + r;
    zs[e] = (b < n && k < MLP_IN) ? mlp_input(md, k, desc[b * MLP_IN + k]) : to_bf16(0.0f);
  }
  __syncthreads();
  mlp_block16(md, zs, h1, h2, yv);
  if (threadIdx.x < 16 && base + threadIdx.x < n)
    dE[base + threadIdx.x] = (double)(yv[threadIdx.x] * md.out_sd + md.out_mu);
}

// ---------------------------------------------------------------------------
// training
// ---------------------------------------------------------------------------
// C[M][N] = sum_k bf16(A(m,k)) bf16(B(k,n)), FP32 accumulation on the MFMA;
// A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn]; one 16x16 tile per
// wave, out-of-range operands read as zero.
__global__ void __launch_bounds__(BLOCK)
    k_gemm_bf16(int M, int N, int K, const float *__restrict__ A, int64_t sam, int64_t sak,
                const float *__restrict__ B, int64_t sbk, int64_t sbn, float *C, int64_t ldc) {
  const int lane = threadIdx.x & 63;
  const int tile = blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6);
  const int tn = (N + 15) / 16, tm = (M + 15) / 16;
  if (tile >= tm * tn) return;  // whole wave leaves together
  const int m0 = (tile / tn) * 16, n0 = (tile % tn) * 16;
  const int r = lane & 15, kb = (lane >> 4) * 8;
  floatx4 c = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 32) {
    bf16x8 a, b;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int k = k0 + kb + q;
      const int mm = m0 + r, nn = n0 + r;
      a[q] = to_bf16((mm < M && k < K) ? A[mm * sam + k * sak] : 0.0f);
      b[q] = to_bf16((nn < N && k < K) ? B[k * sbk + nn * sbn] : 0.0f);
    }
    c = mfma16(a, b, c);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int mm = m0 + (lane >> 4) * 4 + q, nn = n0 + r;
    if (mm < M && nn < N) C[mm * ldc + nn] = c[q];
  }
}

static hipError_t gemm(hipStream_t s, int M, int N, int K, const float *A, int64_t sam,
                       int64_t sak, const float *B, int64_t sbk, int64_t sbn, float *C,
                       int64_t ldc) {
  const int tiles = ((M + 15) / 16) * ((N + 15) / 16);
  k_gemm_bf16<<<(tiles + 3) / 4, BLOCK, 0, s>>>(M, N, K, A, sam, sak, B, sbk, sbn, C, ldc);
  return hipGetLastError();
}

// normalized, bf16-rounded inputs and targets of the batch: samples 0..B-1
// (draw == 0) or Philox-drawn sample indices, with replacement (draw != 0)
__global__ void k_batch(int64_t n, int64_t B, const double *__restrict__ desc,
                        const double *__restrict__ dE, MlpDev md, uint64_t seed, uint64_t step,
                        int draw, float *Z, float *T) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  int64_t src = b;
  if (draw) {
    const U4 r = philox(seed, 0x5EEDull, step, (uint64_t)b, 0, 7);
    src = (int64_t)__umul64hi(r.v[0], (uint64_t)n);
  }
  for (int k = 0; k < MLP_IN; ++k) {
    const float z = (float)((desc[src * MLP_IN + k] - (double)md.mu[k]) / (double)md.sd[k]);
    Z[b * MLP_IN + k] = bf16_round(z);
  }
  T[b] = (float)((dE[src] - (double)md.out_mu) / (double)md.out_sd);
}

// A <- A + bias, H <- bf16(SiLU(A)) over [B][64]
__global__ void k_bias_silu(int64_t B, float *A, const float *__restrict__ bias, float *H) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * MLP_H) return;
  const float a = A[e] + bias[e % MLP_H];
  A[e] = a;
  H[e] = bf16_round(silu(a));
}

// y = b3 + sum_k w3r[k] H2[b][k]; dY = 2 (y - t) / B; per-sample squared error
__global__ void k_out(int64_t B, const float *__restrict__ H2, const float *__restrict__ w3r,
                      const float *__restrict__ b3, const float *__restrict__ T, float *Y,
                      float *dY, double *se) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float acc = b3[0];
  for (int k = 0; k < MLP_H; ++k) acc += w3r[k] * H2[b * MLP_H + k];
  Y[b] = acc;
  const float r = acc - T[b];
  dY[b] = 2.0f * r / (float)B;
  se[b] = (double)r * (double)r;
}

__device__ __forceinline__ float dsilu(float a) {
  const float s = 1.0f / (1.0f + expf(-a));
  return s * (1.0f + a * (1.0f - s));
}

// dA2[b][j] = dY[b] w3r[j] SiLU'(A2[b][j])
__global__ void k_bwd_out(int64_t B, const float *__restrict__ dY, const float *__restrict__ w3r,
                          const float *__restrict__ A2, float *dA2) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * MLP_H) return;
  dA2[e] = dY[e / MLP_H] * w3r[e % MLP_H] * dsilu(A2[e]);
}

// dA1 = dH1 * SiLU'(A1)
__global__ void k_bwd_hidden(int64_t B, const float *__restrict__ dH1, const float *__restrict__ A1,
                             float *dA1) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * MLP_H) return;
  dA1[e] = dH1[e] * dsilu(A1[e]);
}

// out[c] = sum_b X[b][c] (cols columns), and optionally out2[c] = sum_b w[b] X[b][c]
// one thread per column, ascending b (deterministic)
__global__ void k_colsum(int64_t B, int cols, const float *__restrict__ X, const float *__restrict__ w,
                         float *out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float acc = 0.f;
  for (int64_t b = 0; b < B; ++b) acc += (w ? w[b] : 1.0f) * X[b * cols + c];
  out[c] = acc;
}

// fixed-order double sum of v[0..n) into *out, divided by div (one block)
__global__ void k_dsum(int64_t n, const double *__restrict__ v, double *out, double div) {
  __shared__ double s[BLOCK];
  double acc = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += BLOCK) acc = acc + v[k];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int h = BLOCK / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) s[threadIdx.x] = s[threadIdx.x] + s[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0] / div;
}

// Adam on the FP32 master parameters
__global__ void k_adam(float *p, const float *__restrict__ g, float *m1, float *m2, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= MLP_NPARAM) return;
  const float gt = g[t];
  const float a = b1 * m1[t] + (1.0f - b1) * gt;
  const float v = b2 * m2[t] + (1.0f - b2) * gt * gt;
  m1[t] = a;
  m2[t] = v;
  p[t] = p[t] - lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// per-column mean and standard deviation of [n][cols] doubles (fixed order)
__global__ void k_moments(int64_t n, int cols, const double *__restrict__ X, double *out) {
  __shared__ double s1[BLOCK], s2[BLOCK];
  const int c = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += BLOCK) {
    const double v = X[k * cols + c];
    a = a + v;
    b = b + v * v;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int h = BLOCK / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s1[threadIdx.x] = s1[threadIdx.x] + s1[threadIdx.x + h];
      s2[threadIdx.x] = s2[threadIdx.x] + s2[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mean = s1[0] / (double)n;
    const double var = s2[0] / (double)n - mean * mean;
    out[2 * c] = mean;
    out[2 * c + 1] = var > 0.0 ? sqrt(var) : 0.0;
  }
}

// Activations, gradients and loss partials of one batch: the network's own
// buffers (grown on demand) or a fixed workspace.
struct MlpWork {
  float *Z, *T, *A1, *H1, *A2, *H2, *Y, *dY, *dA2, *dH1, *dA1;
  double *red;  // per-sample squared errors [B]
  float *g;     // gradient [4929]
};

// floats of workspace per sample (Z, T, A1, H1, A2, H2, Y, dY, dA2, dH1, dA1)
constexpr int64_t MLP_WORK_PER_SAMPLE = MLP_IN + 1 + 4 * MLP_H + 2 + 3 * MLP_H;

static MlpWork own_work(vcsgc_mlp *m) {
  return MlpWork{m->Z, m->T, m->A1, m->H1, m->A2, m->H2, m->Y, m->dY, m->dA2, m->dH1, m->dA1,
                 m->red, m->g};
}

// Full forward + backward over a batch already in w.Z / w.T; gradient into
// w.g, per-sample squared errors into w.red.  Reads the network's parameters
// only.
static hipError_t mlp_fwd_bwd(const vcsgc_mlp *m, const MlpWork &w, int64_t B, hipStream_t s) {
  const float *p = m->p;
  hipError_t e;
  const int gB = grid_for(B), gBH = grid_for(B * MLP_H);
  // layer 1: A1 = Z W1^T (+ b1), H1 = bf16(SiLU(A1))
  if ((e = gemm(s, (int)B, MLP_H, MLP_IN, w.Z, MLP_IN, 1, p + OFF_W1, 1, MLP_IN, w.A1, MLP_H)))
    return e;
  k_bias_silu<<<gBH, BLOCK, 0, s>>>(B, w.A1, p + OFF_B1, w.H1);
  // layer 2
  if ((e = gemm(s, (int)B, MLP_H, MLP_H, w.H1, MLP_H, 1, p + OFF_W2, 1, MLP_H, w.A2, MLP_H)))
    return e;
  k_bias_silu<<<gBH, BLOCK, 0, s>>>(B, w.A2, p + OFF_B2, w.H2);
  k_out<<<gB, BLOCK, 0, s>>>(B, w.H2, m->w3r, p + OFF_B3, w.T, w.Y, w.dY, w.red);
  // output layer gradients
  k_colsum<<<1, 64, 0, s>>>(B, MLP_H, w.H2, w.dY, w.g + OFF_W3);
  k_colsum<<<1, 64, 0, s>>>(B, 1, w.dY, nullptr, w.g + OFF_B3);
  k_bwd_out<<<gBH, BLOCK, 0, s>>>(B, w.dY, m->w3r, w.A2, w.dA2);
  // layer 2 gradients: dW2 = dA2^T H1, db2, dH1 = dA2 W2
  if ((e = gemm(s, MLP_H, MLP_H, (int)B, w.dA2, 1, MLP_H, w.H1, MLP_H, 1, w.g + OFF_W2, MLP_H)))
    return e;
  k_colsum<<<1, 64, 0, s>>>(B, MLP_H, w.dA2, nullptr, w.g + OFF_B2);
  if ((e = gemm(s, (int)B, MLP_H, MLP_H, w.dA2, MLP_H, 1, p + OFF_W2, MLP_H, 1, w.dH1, MLP_H)))
    return e;
  k_bwd_hidden<<<gBH, BLOCK, 0, s>>>(B, w.dH1, w.A1, w.dA1);
  // layer 1 gradients: dW1 = dA1^T Z, db1
  if ((e = gemm(s, MLP_H, MLP_IN, (int)B, w.dA1, 1, MLP_H, w.Z, MLP_IN, 1, w.g + OFF_W1, MLP_IN)))
    return e;
  k_colsum<<<1, 64, 0, s>>>(B, MLP_H, w.dA1, nullptr, w.g + OFF_B1);
  return hipGetLastError();
}

hipError_t mlp_ensure_cap(vcsgc_mlp *m, int64_t B) {
  if (B <= m->cap) return hipSuccess;
  float **bufs[] = {&m->Z, &m->T, &m->A1, &m->H1, &m->A2, &m->H2, &m->Y, &m->dY,
                    &m->dA2, &m->dH1, &m->dA1};
  const int64_t sizes[] = {B * MLP_IN, B, B * MLP_H, B * MLP_H, B * MLP_H, B * MLP_H, B, B,
                           B * MLP_H, B * MLP_H, B * MLP_H};
  (void)hipStreamSynchronize(m->stream);
  for (int k = 0; k < 11; ++k) {
    if (*bufs[k]) (void)hipFree(*bufs[k]);
    *bufs[k] = nullptr;
    hipError_t e = hipMalloc((void **)bufs[k], sizeof(float) * sizes[k]);
    if (e != hipSuccess) return e;
  }
  if (m->red) (void)hipFree(m->red);
  m->red = nullptr;
  hipError_t e = hipMalloc((void **)&m->red, sizeof(double) * (B + 8));
  if (e != hipSuccess) return e;
  m->cap = B;
  return hipSuccess;
}

hipError_t mlp_grad_batch(vcsgc_mlp *m, const double *desc, const double *dE, int64_t n,
                          double *loss) {
  hipError_t e = mlp_ensure_cap(m, n);
  if (e != hipSuccess) return e;
  MlpDev md = mlp_dev(m);
  k_batch<<<grid_for(n), BLOCK, 0, m->stream>>>(n, n, desc, dE, md, 0, 0, 0, m->Z, m->T);
  if ((e = mlp_fwd_bwd(m, own_work(m), n, m->stream)) != hipSuccess) return e;
  k_dsum<<<1, BLOCK, 0, m->stream>>>(n, m->red, m->red + m->cap, 1.0);
  double h = 0.0;
  e = hipMemcpyAsync(&h, m->red + m->cap, sizeof(double), hipMemcpyDeviceToHost, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (loss) *loss = h / (double)n;
  return e;
}

hipError_t mlp_train(vcsgc_mlp *m, const double *desc, const double *dE, int64_t n,
                     const vcsgc_train_cfg *cfg, vcsgc_train_report *rep) {
  const int64_t B = cfg->batch;
  hipError_t e = mlp_ensure_cap(m, B);
  if (e != hipSuccess) return e;
  const int64_t steps_per_epoch = (n + B - 1) / B;
  const int64_t steps = steps_per_epoch * cfg->epochs;
  MlpDev md = mlp_dev(m);
  double first = -1.0, last = 0.0, acc = 0.0;
  int64_t acc_n = 0;
  for (int64_t st = 0; st < steps; ++st) {
    k_batch<<<grid_for(B), BLOCK, 0, m->stream>>>(n, B, desc, dE, md, cfg->seed, (uint64_t)st, 1,
                                                  m->Z, m->T);
    if ((e = mlp_fwd_bwd(m, own_work(m), B, m->stream)) != hipSuccess) return e;
    m->adam_t += 1;
    const float c1 = 1.0f - powf((float)cfg->beta1, (float)m->adam_t);
    const float c2 = 1.0f - powf((float)cfg->beta2, (float)m->adam_t);
    k_adam<<<grid_for(MLP_NPARAM), BLOCK, 0, m->stream>>>(m->p, m->g, m->m1, m->m2, (float)cfg->lr,
                                                          (float)cfg->beta1, (float)cfg->beta2,
                                                          (float)cfg->eps, c1, c2);
    if ((e = mlp_refresh(m)) != hipSuccess) return e;
    // epoch-end loss of the last batch (one read-back per epoch)
    if ((st + 1) % steps_per_epoch == 0 || st == 0) {
      k_dsum<<<1, BLOCK, 0, m->stream>>>(B, m->red, m->red + m->cap, 1.0);
      double h = 0.0;
      e = hipMemcpyAsync(&h, m->red + m->cap, sizeof(double), hipMemcpyDeviceToHost, m->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
      if (e != hipSuccess) return e;
      h /= (double)B;
      if (first < 0.0) first = h;
      last = h;
      acc += h;
      acc_n += 1;
    }
  }
  if (rep) {
    rep->loss_first = first;
    rep->loss_last = last;
    rep->steps = steps;
  }
  return hipSuccess;
}

hipError_t mlp_forward(vcsgc_mlp *m, const double *desc, int64_t n, double *dE) {
  if (n <= 0) return hipSuccess;
  k_mlp_infer<<<(unsigned)((n + 15) / 16), BLOCK, 0, m->stream>>>(mlp_dev(m), n, desc, dE);
  return hipGetLastError();
}

hipError_t mlp_fit_normalization(vcsgc_mlp *m, const double *desc, const double *dE, int64_t n) {
  hipError_t e = mlp_ensure_cap(m, 1);
  if (e != hipSuccess) return e;
  double *st = nullptr;
  e = hipMalloc((void **)&st, sizeof(double) * 22);
  if (e != hipSuccess) return e;
  k_moments<<<MLP_IN, BLOCK, 0, m->stream>>>(n, MLP_IN, desc, st);
  k_moments<<<1, BLOCK, 0, m->stream>>>(n, 1, dE, st + 20);
  double h[22];
  e = hipMemcpyAsync(h, st, sizeof(h), hipMemcpyDeviceToHost, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  (void)hipFree(st);
  if (e != hipSuccess) return e;
  for (int k = 0; k < MLP_IN; ++k) {
    m->mu[k] = (float)h[2 * k];
    m->sd[k] = h[2 * k + 1] > 1e-6 ? (float)h[2 * k + 1] : 1.0f;
  }
  m->out_mu = (float)h[20];
  m->out_sd = h[21] > 1e-9 ? (float)h[21] : 1.0f;
  return hipSuccess;
}

}  // namespace vc

// ---------------------------------------------------------------------------
// C ABI of the network
// ---------------------------------------------------------------------------
namespace {

vcsgc_status mfail(vcsgc_mlp *m, hipError_t e, const char *where) {
  if (m) m->err = std::string(where) + ": " + hipGetErrorString(e);
  return VCSGC_E_DEVICE;
}

// deterministic initial weights: uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)),
// zero biases, from a 64-bit linear congruential stream
void init_params(uint64_t seed, std::vector<float> &p) {
  uint64_t x = seed * 6364136223846793005ull + 1442695040888963407ull;
  auto next = [&]() {
    x = x * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(x >> 11) * 0x1p-53;
  };
  p.assign(vc::MLP_NPARAM, 0.0f);
  const double s1 = 1.0 / std::sqrt(10.0), s2 = 1.0 / std::sqrt(64.0);
  for (int k = 0; k < 640; ++k) p[vc::OFF_W1 + k] = (float)((2.0 * next() - 1.0) * s1);
  for (int k = 0; k < 4096; ++k) p[vc::OFF_W2 + k] = (float)((2.0 * next() - 1.0) * s2);
  for (int k = 0; k < 64; ++k) p[vc::OFF_W3 + k] = (float)((2.0 * next() - 1.0) * s2);
}

}  // namespace

extern "C" {

vcsgc_status vcsgc_mlp_create(uint64_t seed, hipStream_t stream, vcsgc_mlp **out) {
  if (!out) return VCSGC_E_INVALID_ARG;
  vcsgc_mlp *m = new vcsgc_mlp();
  (void)hipGetDevice(&m->device);
  m->stream = stream;
  for (int k = 0; k < 10; ++k) {
    m->mu[k] = 0.f;
    m->sd[k] = 1.f;
  }
  hipError_t e = hipMalloc((void **)&m->p, sizeof(float) * vc::MLP_NPARAM);
  if (e == hipSuccess) e = hipMalloc((void **)&m->g, sizeof(float) * vc::MLP_NPARAM);
  if (e == hipSuccess) e = hipMalloc((void **)&m->m1, sizeof(float) * vc::MLP_NPARAM);
  if (e == hipSuccess) e = hipMalloc((void **)&m->m2, sizeof(float) * vc::MLP_NPARAM);
  if (e == hipSuccess) e = hipMalloc((void **)&m->w1b, sizeof(__bf16) * 64 * 32);
  if (e == hipSuccess) e = hipMalloc((void **)&m->w2b, sizeof(__bf16) * 64 * 64);
  if (e == hipSuccess) e = hipMalloc((void **)&m->w3r, sizeof(float) * 64);
  std::vector<float> p;
  init_params(seed, p);
  if (e == hipSuccess)
    e = hipMemcpy(m->p, p.data(), sizeof(float) * vc::MLP_NPARAM, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemsetAsync(m->m1, 0, sizeof(float) * vc::MLP_NPARAM, stream);
  if (e == hipSuccess) e = hipMemsetAsync(m->m2, 0, sizeof(float) * vc::MLP_NPARAM, stream);
  if (e == hipSuccess) e = vc::mlp_refresh(m);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    vcsgc_mlp_destroy(m);
    return e == hipErrorOutOfMemory ? VCSGC_E_OUT_OF_MEMORY : VCSGC_E_DEVICE;
  }
  *out = m;
  return VCSGC_OK;
}

vcsgc_status vcsgc_mlp_destroy(vcsgc_mlp *m) {
  if (!m) return VCSGC_OK;
  (void)hipStreamSynchronize(m->stream);
  void *ptrs[] = {m->p, m->g, m->m1, m->m2, m->w1b, m->w2b, m->w3r, m->Z, m->T, m->A1, m->H1,
                  m->A2, m->H2, m->Y, m->dY, m->dA2, m->dH1, m->dA1, m->red};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  delete m;
  return VCSGC_OK;
}

vcsgc_status vcsgc_mlp_set_params(vcsgc_mlp *m, const float *params, const float *mu,
                                  const float *sd, float out_mu, float out_sd) {
  if (!m || !params || !mu || !sd || !(out_sd > 0.f)) return VCSGC_E_INVALID_ARG;
  for (int k = 0; k < 10; ++k)
    if (!(sd[k] > 0.f)) return VCSGC_E_INVALID_ARG;
  hipError_t e = hipMemcpy(m->p, params, sizeof(float) * vc::MLP_NPARAM, hipMemcpyHostToDevice);
  if (e != hipSuccess) return mfail(m, e, "set_params");
  for (int k = 0; k < 10; ++k) {
    m->mu[k] = mu[k];
    m->sd[k] = sd[k];
  }
  m->out_mu = out_mu;
  m->out_sd = out_sd;
  e = vc::mlp_refresh(m);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  return e == hipSuccess ? VCSGC_OK : mfail(m, e, "set_params");
}

vcsgc_status vcsgc_mlp_get_params(vcsgc_mlp *m, float *params, float *mu, float *sd,
                                  float *out_mu, float *out_sd) {
  if (!m) return VCSGC_E_INVALID_ARG;
  if (params) {
    hipError_t e = hipStreamSynchronize(m->stream);
    if (e == hipSuccess)
      e = hipMemcpy(params, m->p, sizeof(float) * vc::MLP_NPARAM, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return mfail(m, e, "get_params");
  }
  for (int k = 0; k < 10; ++k) {
    if (mu) mu[k] = m->mu[k];
    if (sd) sd[k] = m->sd[k];
  }
  if (out_mu) *out_mu = m->out_mu;
  if (out_sd) *out_sd = m->out_sd;
  return VCSGC_OK;
}

vcsgc_status vcsgc_mlp_fit_normalization(vcsgc_mlp *m, const double *desc_dev,
                                         const double *dE_dev, int64_t n) {
  if (!m || !desc_dev || !dE_dev || n < 2) return VCSGC_E_INVALID_ARG;
  hipError_t e = vc::mlp_fit_normalization(m, desc_dev, dE_dev, n);
  return e == hipSuccess ? VCSGC_OK : mfail(m, e, "fit_normalization");
}

vcsgc_status vcsgc_mlp_train(vcsgc_mlp *m, const double *desc_dev, const double *dE_dev,
                             int64_t n, const vcsgc_train_cfg *cfg, vcsgc_train_report *report) {
  if (!m || !desc_dev || !dE_dev || !cfg || n < 1 || cfg->epochs < 0 || cfg->batch < 1 ||
      cfg->batch > (1 << 22) || !(cfg->lr > 0.0) || !(cfg->beta1 >= 0.0 && cfg->beta1 < 1.0) ||
      !(cfg->beta2 >= 0.0 && cfg->beta2 < 1.0) || !(cfg->eps > 0.0))
    return VCSGC_E_INVALID_ARG;
  hipError_t e = vc::mlp_train(m, desc_dev, dE_dev, n, cfg, report);
  return e == hipSuccess ? VCSGC_OK : mfail(m, e, "train");
}

vcsgc_status vcsgc_mlp_forward(vcsgc_mlp *m, const double *desc_dev, int64_t n, double *dE_dev) {
  if (!m || n < 0 || (n > 0 && (!desc_dev || !dE_dev))) return VCSGC_E_INVALID_ARG;
  hipError_t e = vc::mlp_forward(m, desc_dev, n, dE_dev);
  return e == hipSuccess ? VCSGC_OK : mfail(m, e, "forward");
}

vcsgc_status vcsgc_mlp_grad(vcsgc_mlp *m, const double *desc_dev, const double *dE_dev, int64_t n,
                            float *grad_host, double *loss) {
  if (!m || !desc_dev || !dE_dev || n < 1 || n > (1 << 22)) return VCSGC_E_INVALID_ARG;
  hipError_t e = vc::mlp_grad_batch(m, desc_dev, dE_dev, n, loss);
  if (e == hipSuccess && grad_host)
    e = hipMemcpy(grad_host, m->g, sizeof(float) * vc::MLP_NPARAM, hipMemcpyDeviceToHost);
  return e == hipSuccess ? VCSGC_OK : mfail(m, e, "grad");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free gradient (vcsgc_mlp_grad_noalloc).  The batch's workspace
// (activations, back-propagated errors and per-sample squared errors of at
// most VCSGC_NOALLOC_MAX_SAMPLES samples) is a fixed device array, so the
// call allocates nothing on any path; outputs go to caller device memory and
// nothing is read back.  The array's device address is looked up once per
// device (hipGetSymbolAddress) and only that address reaches the kernels.
// Every kernel of the pass writes its whole output, so nothing needs clearing
// between calls; calls that overlap on one device share the array and race.
// ---------------------------------------------------------------------------
#include <mutex>

namespace vc {

constexpr int64_t NA_MAX = VCSGC_NOALLOC_MAX_SAMPLES;
constexpr size_t NA_FLOAT_BYTES = sizeof(float) * (size_t)(NA_MAX * MLP_WORK_PER_SAMPLE);
constexpr size_t NA_BYTES = NA_FLOAT_BYTES + sizeof(double) * (size_t)NA_MAX;
static_assert(NA_FLOAT_BYTES % 256 == 0, "double area aligned");

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

constexpr int NA_DEVICES = 64;
static void *g_scratch[NA_DEVICES] = {};
static std::mutex g_scratch_mu;

// device address of `scratch` on `dev` (looked up once per device)
static hipError_t scratch_address(int dev, unsigned char **out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    g_scratch[dev] = ptr;
  }
  *out = (unsigned char *)g_scratch[dev];
  return hipSuccess;
}

static MlpWork fixed_work(unsigned char *base, int64_t B, float *grad) {
  float *f = (float *)base;
  MlpWork w;
  float **bufs[] = {&w.Z, &w.T, &w.A1, &w.H1, &w.A2, &w.H2, &w.Y, &w.dY, &w.dA2, &w.dH1, &w.dA1};
  const int64_t per[] = {MLP_IN, 1, MLP_H, MLP_H, MLP_H, MLP_H, 1, 1, MLP_H, MLP_H, MLP_H};
  for (int k = 0; k < 11; ++k) {
    *bufs[k] = f;
    f += per[k] * B;
  }
  w.red = (double *)(base + NA_FLOAT_BYTES);
  w.g = grad;
  return w;
}

}  // namespace vc

extern "C" vcsgc_status vcsgc_mlp_grad_noalloc(const vcsgc_mlp *m, const double *desc_dev,
                                               const double *dE_dev, int64_t n, float *grad_dev,
                                               double *loss_dev) {
  if (!m || !desc_dev || !dE_dev || !grad_dev || !loss_dev) return VCSGC_E_INVALID_ARG;
  if (n < 1 || n > VCSGC_NOALLOC_MAX_SAMPLES) return VCSGC_E_INVALID_ARG;
  if (m->device < 0 || m->device >= vc::NA_DEVICES) return VCSGC_E_INVALID_ARG;
  unsigned char *base = nullptr;
  hipError_t e = vc::scratch_address(m->device, &base);
  if (e != hipSuccess) return VCSGC_E_DEVICE;
  const vc::MlpWork w = vc::fixed_work(base, n, grad_dev);
  const vc::MlpDev md = vc::mlp_dev(m);
  vc::k_batch<<<vc::grid_for(n), vc::BLOCK, 0, m->stream>>>(n, n, desc_dev, dE_dev, md, 0, 0, 0,
                                                            w.Z, w.T);
  e = vc::mlp_fwd_bwd(m, w, n, m->stream);
  if (e != hipSuccess) return VCSGC_E_DEVICE;
  vc::k_dsum<<<1, vc::BLOCK, 0, m->stream>>>(n, w.red, loss_dev, (double)n);
  return hipGetLastError() == hipSuccess ? VCSGC_OK : VCSGC_E_DEVICE;
}
