// Kernels of the MLP surrogate that ranks greedy candidates (not part of the paper's
// method; it replaces most full sweeps of the indicator in Alg. 4).
//
// Network P -> H -> H -> 1 with exact-erf GELU, MSE loss on log10(indicator), Adam.
// Products run on MFMA with FP32 accumulation; in BF16 mode both operands are rounded
// to BF16 (nearest even) as they are loaded, in FP32 mode they stay FP32.
#include <hip/hip_runtime.h>

#include "internal.h"
#include "mlp.h"

namespace rb {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float gelu_f(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float dgelu_f(float z) {
  const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * z * z);
  return cdf + z * pdf;
}

// C[m][n] = sum_k A[m][k] B[k][n] for m < M, n < N (A at A + m*sam + k*sak, B at
// B + k*sbk + n*sbn), one wavefront per 16x16 tile of C, four tiles per block along M.
// Epilogues: EPI_STORE: C = acc (+ bias[n]); EPI_GELU: Z = acc + bias[n], C = Z,
// C2 = gelu(Z); EPI_DGELU: C = acc * gelu'(aux[m*ldaux + n]).
enum { EPI_STORE = 0, EPI_GELU = 1, EPI_DGELU = 2 };

template <bool BF16, int EPI>
__global__ __launch_bounds__(256) void k_mm(int M, int N, int K, const float* __restrict__ A,
                                            int sam, int sak, const float* __restrict__ B,
                                            int sbk, int sbn, const float* __restrict__ bias,
                                            float* __restrict__ C, int ldc, float* __restrict__ C2,
                                            const float* __restrict__ aux, int ldaux) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = (blockIdx.x * 4 + wave) * 16;
  const int n0 = blockIdx.y * 16;
  if (m0 >= M) return;
  const int r = lane & 15, g = lane >> 4;
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  const int am = m0 + r, bn = n0 + r;
  if constexpr (BF16) {
    for (int k0 = 0; k0 < K; k0 += 16) {
      shortx4 a, b;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = k0 + 4 * g + i;
        const float av = (am < M && k < K) ? A[(size_t)am * sam + (size_t)k * sak] : 0.f;
        const float bv = (bn < N && k < K) ? B[(size_t)k * sbk + (size_t)bn * sbn] : 0.f;
        a[i] = (short)rbk::f32_to_bf16_rne(av);
        b[i] = (short)rbk::f32_to_bf16_rne(bv);
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
  } else {
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int k = k0 + g;
      const float a = (am < M && k < K) ? A[(size_t)am * sam + (size_t)k * sak] : 0.f;
      const float b = (bn < N && k < K) ? B[(size_t)k * sbk + (size_t)bn * sbn] : 0.f;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
  }
  const int n = n0 + r;
  if (n >= N) return;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + 4 * g + i;
    if (m >= M) continue;
    float v = acc[i];
    if (EPI == EPI_DGELU) {
      v *= dgelu_f(aux[(size_t)m * ldaux + n]);
      C[(size_t)m * ldc + n] = v;
    } else {
      if (bias) v += bias[n];
      C[(size_t)m * ldc + n] = v;
      if (EPI == EPI_GELU) C2[(size_t)m * ldc + n] = gelu_f(v);
    }
  }
}

static void mm(bool bf16, int epi, int M, int N, int K, const float* A, int sam, int sak,
               const float* B, int sbk, int sbn, const float* bias, float* C, int ldc, float* C2,
               const float* aux, int ldaux, hipStream_t s) {
  const dim3 grid((M + 63) / 64, (N + 15) / 16);
#define MM(BF, E)                                                                             \
  hipLaunchKernelGGL((k_mm<BF, E>), grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, \
                     bias, C, ldc, C2, aux, ldaux)
  if (bf16) {
    if (epi == EPI_STORE) MM(true, EPI_STORE);
    else if (epi == EPI_GELU) MM(true, EPI_GELU);
    else MM(true, EPI_DGELU);
  } else {
    if (epi == EPI_STORE) MM(false, EPI_STORE);
    else if (epi == EPI_GELU) MM(false, EPI_GELU);
    else MM(false, EPI_DGELU);
  }
#undef MM
}

// out[n] = sum_m G[m][n] (fixed order)
__global__ void k_colsum(const float* __restrict__ G, int M, int N, int ld, float* __restrict__ out) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += G[(size_t)m * ld + n];
  out[n] = s;
}

// loss = mean (out - y)^2 and g[m] = 2 (out_m - y_m) / M; one block of 256 threads
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ out,
                                             const float* __restrict__ y, int M,
                                             float* __restrict__ g, float* __restrict__ loss) {
  __shared__ float sh[256];
  float s = 0.f;
  for (int m = threadIdx.x; m < M; m += 256) {
    const float d = out[m] - y[m];
    g[m] = 2.0f * d / (float)M;
    s += d * d;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = sh[0] / (float)M;
}

// Adam with bias correction on FP32 masters
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.0f - b1) * gi;
  const float b = b2 * m2[i] + (1.0f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  p[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

// features u = (log10 mu - mid) / half, FP32
__global__ void k_features(const double* __restrict__ mu, int count, double mid, double half,
                           float* __restrict__ u) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) u[i] = (float)((log10(mu[i]) - mid) / half);
}

// gathers rows of X (ld P) and targets into a contiguous minibatch
__global__ void k_gather(const float* __restrict__ X, const float* __restrict__ Y, int P,
                         const int* __restrict__ idx, int m, float* __restrict__ Xb,
                         float* __restrict__ Yb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int s = idx[i];
  for (int k = 0; k < P; ++k) Xb[(size_t)i * P + k] = X[(size_t)s * P + k];
  if (Y) Yb[i] = Y[s];
}

// ---- host-side network driver ------------------------------------------------------------
MLP::MLP(int P_, int H_, bool bf16_, int max_rows, hipStream_t s)
    : P(P_), H(H_), bf16(bf16_), rows(max_rows), st(s) {
  count = H * P + H * H + 3 * H + 1;
  params.alloc(sizeof(float) * count);
  grads.alloc(sizeof(float) * count);
  m1.alloc(sizeof(float) * count);
  m2.alloc(sizeof(float) * count);
  const size_t act = sizeof(float) * (size_t)rows * H;
  Z1.alloc(act); A1.alloc(act); Z2.alloc(act); A2.alloc(act);
  G1.alloc(act); G2.alloc(act);
  out.alloc(sizeof(float) * rows);
  gout.alloc(sizeof(float) * rows);
  loss.alloc(sizeof(float) * 4);
}

void MLP::set_params(const float* host) {
  RB_HIP(hipMemcpyAsync(params.p, host, sizeof(float) * count, hipMemcpyHostToDevice, st));
  RB_HIP(hipMemsetAsync(m1.p, 0, sizeof(float) * count, st));
  RB_HIP(hipMemsetAsync(m2.p, 0, sizeof(float) * count, st));
  t = 0;
}
void MLP::get_params(float* host) {
  RB_HIP(hipMemcpyAsync(host, params.p, sizeof(float) * count, hipMemcpyDeviceToHost, st));
  RB_HIP(hipStreamSynchronize(st));
}

// forward of m rows of X [m][P] (device); result in out[0..m)
void MLP::forward(const float* X, int m) {
  RB_REQUIRE(m <= rows, RB_EINVAL, "MLP batch larger than its workspace");
  const float* p = params.as<float>();
  const float *W1 = p + oW1(), *b1 = p + ob1(), *W2 = p + oW2(), *b2 = p + ob2(), *w3 = p + ow3(),
              *b3 = p + ob3();
  // Z1 = X W1^T + b1, A1 = gelu(Z1): B[k][n] = W1[n][k]
  mm(bf16, EPI_GELU, m, H, P, X, P, 1, W1, 1, P, b1, Z1.as<float>(), H, A1.as<float>(), nullptr, 0,
     st);
  mm(bf16, EPI_GELU, m, H, H, A1.as<float>(), H, 1, W2, 1, H, b2, Z2.as<float>(), H,
     A2.as<float>(), nullptr, 0, st);
  mm(bf16, EPI_STORE, m, 1, H, A2.as<float>(), H, 1, w3, 1, H, b3, out.as<float>(), 1, nullptr,
     nullptr, 0, st);
}

// loss and gradients of the mean squared error on m rows (targets y, device)
void MLP::backward(const float* X, const float* y, int m) {
  forward(X, m);
  float* gp = grads.as<float>();
  const float* p = params.as<float>();
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, st, out.as<float>(), y, m, gout.as<float>(),
                     loss.as<float>());
  // output layer: g_w3[k] = sum_m g_out[m] A2[m][k]; g_b3 = sum g_out
  mm(bf16, EPI_STORE, 1, H, m, gout.as<float>(), 0, 1, A2.as<float>(), H, 1, nullptr, gp + ow3(),
     H, nullptr, nullptr, 0, st);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(64), 0, st, gout.as<float>(), m, 1, 1, gp + ob3());
  // G2 = (g_out w3) * gelu'(Z2)   (outer product, K = 1)
  mm(bf16, EPI_DGELU, m, H, 1, gout.as<float>(), 1, 1, p + ow3(), H, 1, nullptr, G2.as<float>(), H,
     nullptr, Z2.as<float>(), H, st);
  // g_W2[o][k] = sum_m G2[m][o] A1[m][k]; g_b2 = colsum G2
  mm(bf16, EPI_STORE, H, H, m, G2.as<float>(), 1, H, A1.as<float>(), H, 1, nullptr, gp + oW2(), H,
     nullptr, nullptr, 0, st);
  hipLaunchKernelGGL(k_colsum, dim3((H + 63) / 64), dim3(64), 0, st, G2.as<float>(), m, H, H,
                     gp + ob2());
  // G1 = (G2 W2) * gelu'(Z1): B[k][n] = W2[k][n]
  mm(bf16, EPI_DGELU, m, H, H, G2.as<float>(), H, 1, p + oW2(), H, 1, nullptr, G1.as<float>(), H,
     nullptr, Z1.as<float>(), H, st);
  // g_W1[o][k] = sum_m G1[m][o] X[m][k]; g_b1 = colsum G1
  mm(bf16, EPI_STORE, H, P, m, G1.as<float>(), 1, H, X, P, 1, nullptr, gp + oW1(), P, nullptr,
     nullptr, 0, st);
  hipLaunchKernelGGL(k_colsum, dim3((H + 63) / 64), dim3(64), 0, st, G1.as<float>(), m, H, H,
                     gp + ob1());
}

void MLP::adam(double lr) {
  ++t;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3((count + 255) / 256), dim3(256), 0, st, params.as<float>(),
                     grads.as<float>(), m1.as<float>(), m2.as<float>(), count, (float)lr, b1, b2,
                     eps, c1, c2);
}

float MLP::last_loss() {
  float l = 0.f;
  RB_HIP(hipMemcpyAsync(&l, loss.p, sizeof(float), hipMemcpyDeviceToHost, st));
  RB_HIP(hipStreamSynchronize(st));
  return l;
}

void launch_features(const double* mu, int count, double mid, double half, float* u,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_features, dim3((count + 255) / 256), dim3(256), 0, s, mu, count, mid, half,
                     u);
}
void launch_gather(const float* X, const float* Y, int P, const int* idx, int m, float* Xb,
                   float* Yb, hipStream_t s) {
  hipLaunchKernelGGL(k_gather, dim3((m + 255) / 256), dim3(256), 0, s, X, Y, P, idx, m, Xb, Yb);
}

// ---- top-K selection --------------------------------------------------------------------
// The K largest of v[0..M) among entries with excluded[m] == 0, as a set of indices
// (ties at the threshold resolved towards lower indices).  One block of 1024 threads:
// the threshold is found by a radix select on the order-preserving integer image of
// the float keys, 8 bits at a time; then an ordered compaction writes the winners.
__device__ __forceinline__ uint32_t fkey(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ __launch_bounds__(1024) void k_topk(const float* __restrict__ v,
                                               const int* __restrict__ excluded, int M, int K,
                                               int* __restrict__ out, int* __restrict__ out_count) {
  __shared__ unsigned hist[256];
  __shared__ uint32_t prefix_sh, want_sh;
  __shared__ int cnt_gt[1024], cnt_eq[1024];
  const int tid = threadIdx.x;
  uint32_t prefix = 0, pmask = 0;
  uint32_t want = (uint32_t)K;  // how many of the remaining candidates to take
  int avail = 0;
  for (int m = tid; m < M; m += 1024) avail += excluded[m] ? 0 : 1;
  // total available
  cnt_gt[tid] = avail;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (tid < off) cnt_gt[tid] += cnt_gt[tid + off];
    __syncthreads();
  }
  const int total = cnt_gt[0];
  __syncthreads();
  if ((int)want > total) want = (uint32_t)total;
  for (int shift = 24; shift >= 0 && want > 0; shift -= 8) {
    if (tid < 256) hist[tid] = 0;
    __syncthreads();
    for (int m = tid; m < M; m += 1024) {
      if (excluded[m]) continue;
      const uint32_t k = fkey(v[m]);
      if ((k & pmask) == prefix) atomicAdd(&hist[(k >> shift) & 0xffu], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      uint32_t acc = 0;
      int b = 255;
      for (; b > 0; --b) {
        if (acc + hist[b] >= want) break;
        acc += hist[b];
      }
      prefix_sh = prefix | ((uint32_t)b << shift);
      want_sh = want - acc;
    }
    __syncthreads();
    prefix = prefix_sh;
    want = want_sh;
    pmask |= 0xffu << shift;
    __syncthreads();
  }
  // threshold key = prefix; take every key > prefix and the first `want` equal ones
  const int per = (M + 1023) / 1024;
  const int lo = tid * per, hi = min(M, lo + per);
  int gt = 0, eq = 0;
  for (int m = lo; m < hi; ++m) {
    if (excluded[m]) continue;
    const uint32_t k = fkey(v[m]);
    if (k > prefix) ++gt;
    else if (k == prefix) ++eq;
  }
  cnt_gt[tid] = gt;
  cnt_eq[tid] = eq;
  __syncthreads();
  if (tid == 0) {  // exclusive scans (serial: 1024 entries)
    int sg = 0, se = 0;
    for (int i = 0; i < 1024; ++i) {
      const int a = cnt_gt[i], b = cnt_eq[i];
      cnt_gt[i] = sg;
      cnt_eq[i] = se;
      sg += a;
      se += b;
    }
    *out_count = (total == 0 || K == 0) ? 0 : sg + (int)min((uint32_t)se, want);
    prefix_sh = (uint32_t)sg;  // number of strictly greater keys
  }
  __syncthreads();
  const int n_gt = (int)prefix_sh;
  if (total == 0 || K == 0) return;
  int og = cnt_gt[tid], oe = cnt_eq[tid];
  for (int m = lo; m < hi; ++m) {
    if (excluded[m]) continue;
    const uint32_t k = fkey(v[m]);
    if (k > prefix) {
      out[og++] = m;
    } else if (k == prefix) {
      if ((uint32_t)oe < want) out[n_gt + oe] = m;
      ++oe;
    }
  }
}

void launch_topk(const float* v, const int* excluded, int M, int K, int* out, int* out_count,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_topk, dim3(1), dim3(1024), 0, s, v, excluded, M, K, out, out_count);
}

}  // namespace rb
