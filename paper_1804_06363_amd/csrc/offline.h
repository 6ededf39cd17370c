// Offline greedy state shared by the plain greedy and the surrogate-ranked greedy.
#pragma once

#include <memory>
#include <vector>

#include "internal.h"

namespace rb {

struct GreedyState {
  rb_ctx* ctx;
  const rb_problem* prob;
  rb_greedy_opts opt;
  int M;
  int a_ld = 16;
  std::vector<double> theta_h, phi_h;
  DevBuf theta_d, phi_d;
  DevBuf coeffs;    // [M][a_ld] reduced coefficients a(mu)
  DevBuf ind, l1;   // [M]
  DevBuf cstatus;   // [M]
  DevBuf excluded;  // [M]
  DevBuf amax;      // argmax output (value, index, nan flag)
  DevBuf w;         // snapshot / new basis vector (storage order)
  DevBuf part;
  std::vector<int> excl_h;
  std::vector<double> ind_h;  // last indicator of every candidate (-inf: never evaluated)
  std::unique_ptr<rb_basis> bs;
  double fnorm2 = 1.0;
  int64_t true_evals = 0;
  int full_sweeps = 0;

  GreedyState(rb_ctx* c, const rb_problem* p, const rb_greedy_opts& o, int64_t M,
              const double* theta, const double* phi);
  // starts from a copy of an existing basis (at most opt.n_max columns) and its reduced
  // operators instead of an empty one
  void adopt(const rb_basis* src);
  double norm(const double* v);
  int snapshot(int mu);
  bool orthonormalize_append();
  void sweep(const std::vector<int>& idx);
  int pick(double* value);
};

// MLP-ranked greedy step (mlp.cpp): returns the next pick (or -1) and its indicator.
struct Surrogate {
  GreedyState& gs;
  int P;
  double last_loss = 0.0;
  int fallbacks = 0;  // steps whose ranking check failed (full sweep instead)
  // what the latest step did: its short list (top-K in increasing index order, then the
  // exploration draws in draw order), whether it swept every candidate and whether the
  // ranking check failed
  std::vector<int> last_topk, last_explore;
  bool last_full = false, last_fallback = false;
  struct Impl;
  std::unique_ptr<Impl> impl;
  Surrogate(GreedyState& g, const double* mu, int P);
  ~Surrogate();
  int step(int greedy_step, double* value);
  // state of a surrogate in the middle of a greedy: FP32 master weights (Adam moments
  // reset), replay buffer entries (candidate, target, step) and the counter position
  void set_state(const float* params, int nbuf, const int32_t* idx, const float* target,
                 const int32_t* step, uint64_t counter);
  void get_params(float* params);
  uint64_t counter() const;
  int param_count() const;
};

}  // namespace rb
