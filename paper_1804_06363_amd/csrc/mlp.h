// MLP surrogate network on the GPU (P -> H -> H -> 1, GELU), see mlp.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace rb {

struct MLP {
  int P, H;
  bool bf16;
  int rows;  // largest batch the activation buffers hold
  hipStream_t st;
  int count = 0;  // number of parameters
  int t = 0;      // Adam step
  DevBuf params, grads, m1, m2;
  DevBuf Z1, A1, Z2, A2, G1, G2, out, gout, loss;
  // packed parameter offsets: W1 [H][P], b1 [H], W2 [H][H], b2 [H], w3 [H], b3 [1]
  int oW1() const { return 0; }
  int ob1() const { return H * P; }
  int oW2() const { return H * P + H; }
  int ob2() const { return H * P + H + H * H; }
  int ow3() const { return H * P + 2 * H + H * H; }
  int ob3() const { return H * P + 3 * H + H * H; }

  MLP(int P, int H, bool bf16, int max_rows, hipStream_t s);
  void set_params(const float* host);  // also resets Adam
  void get_params(float* host);
  void forward(const float* X, int m);                   // -> out
  void backward(const float* X, const float* y, int m);  // -> grads, loss
  void adam(double lr);
  float last_loss();
};

void launch_features(const double* mu, int count, double mid, double half, float* u,
                     hipStream_t s);
void launch_gather(const float* X, const float* Y, int P, const int* idx, int m, float* Xb,
                   float* Yb, hipStream_t s);
void launch_topk(const float* v, const int* excluded, int M, int K, int* out, int* out_count,
                 hipStream_t s);

// SplitMix64 used as a counter-based generator: value(seed, i) = mix(seed + (i+1) * gamma).
inline uint64_t splitmix64(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
inline double uniform01(uint64_t seed, uint64_t i) {
  return (double)(splitmix64(seed, i) >> 11) * (1.0 / 9007199254740992.0);
}

}  // namespace rb
