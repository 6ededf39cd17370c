// Batched online solver: RBCG (Alg. 3), RBI (Alg. 2) and plain CG over B queries of
// one problem and one basis.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"

namespace rb {

struct BatchSolver {
  rb_ctx* ctx;
  const rb_problem* prob;
  const rb_basis* basis;  // may be null (CG, or n = 0)
  rb_solve_opts opt;
  int B = 0;
  int n = 0;        // basis columns used (max over queries)
  int e_ld = 16;    // row stride of e
  const int pt = 4;  // nodes per thread of the init/dot kernels (matches stencil_chunks)
  int cN = 1;        // partial-sum chunks of an all-node pass
  Segs gsegs, jsegs;  // y^T r partial segments: per colour sweep / one whole-vector pass
  int pstride = 1;             // per-query stride of the partial-sum arrays
  bool y32 = false;            // y stored in FP32
  bool adaptive = false;       // adaptive basis size (opt.adapt_gamma > 0)
  int rrows = 0;               // rows allocated for r (padded for the projection)
  ProjPlan plan;
  const void* Wsh = nullptr;   // basis in the preconditioner's precision

  // device buffers (views of the context's workspace)
  Buf theta_d, scale_d, nuse_d, ones_d, coef, L, e64, e32, projpart;
  // host copies of the per-query inputs (uploaded by prepare())
  std::vector<double> theta_h, phi_h, sc_h;
  std::vector<int> nu_h;
  Buf qlist;  // active queries in increasing order, then their count (batched coarse step)
  Buf x, r0, r1, p0, p1, y, z;
  Buf xc;  // RBCG / CG: x-updates since the last true-residual check (folded into x there)
  // RBCG with y in FP32 on stencil grids: an FP32 copy of the current r (same rows as r0),
  // written wherever r is; read by the projection and the sweeps without dot products
  bool use_r32 = false;
  bool pair_x = false;  // pass B updates x every second iteration, for two iterations
  Buf r32;
  // fused red-black sweep (3D grids with nx <= 255, one forward sweep): the coarse
  // correction goes to zs (black half) and one launch writes y from it
  bool fused_ok = false;
  Buf zs;
  Segs fsegs;
  bool fused() const { return fused_ok && tc.kind_gs == 3; }
  Buf part_m, part_m2, part_r0, part_r1;
  Buf qbuf;  // QState arrays
  QState q{};
  const double* f_base = nullptr;  // right-hand side term(s), storage order
  int64_t f_ld = 0;                // 0: one shared term scaled per query
  Buf fb, phi_d;                   // f_b = sum_r phi_br f_r when R > 1, and phi
  TuneConfig tc;                    // tile choices of this solve
  std::string tune_key;
  hipGraphExec_t graph = nullptr;
  int graph_parity = 0;

  hipStream_t stream_;
  Workspace* ws_;
  Buf get_ws(int slot, size_t bytes) { return ws_->get(slot, bytes, stream_); }

  // stream / workspace default to the context's
  BatchSolver(rb_ctx* c, const rb_problem* p, const rb_basis* b, const rb_solve_opts& o, int B_,
              const double* theta, const double* phi, const int* n_use,
              hipStream_t stream = nullptr, Workspace* ws = nullptr);
  ~BatchSolver();

  hipStream_t s() const { return stream_; }
  // uploads and per-query initial state (start() calls it; single-step users call it
  // after construction)
  void prepare();
  int64_t ld() const { return prob->ld; }
  // RBCG / CG
  void init_cg();
  void iterate_cg(int k);
  // rc (nullable): the FP32 copy of r
  void precondition(const double* r, const double* r_old, const float* rc = nullptr);
  const Segs& dot_segs() const;
  // RBI
  void init_rbi();
  void iterate_rbi(int k);
  // driver: run() = start(); do fill(); while (poll()); finish().  On large grids one
  // chunk runs while the host reads the previous one's flags.
  void run();
  void start();
  void issue(int iters);
  void fill();  // issues chunks until depth_ are in flight or no iterations are left
  // waits for the oldest chunk in flight; true while its flags show active queries and
  // iterations are left (false when no chunk is in flight)
  bool poll();
  bool more() const { return k_ < limit_; }  // iterations left to issue
  void finish();
  int k_ = 0, limit_ = 0, chunk_ = 0, depth_ = 1;
  bool fixed_ = false, rbi_ = false;
  // Chunks of iterations in flight (at most depth_ <= 2): each issue() copies the active flags
  // after its chunk into its own pinned host buffer and records an event, so the host
  // queues the next chunk before it looks at the previous one's flags.
  int* hflags_[2] = {nullptr, nullptr};
  hipEvent_t hev_[2] = {nullptr, nullptr};
  int kdone_[2] = {0, 0};  // k_ at the end of each chunk in flight
  int issued_ = 0, polled_ = 0;
  void final_true_residual();
  void gather(double* x_user_nat, int64_t user_ld, std::vector<rb_query_stats>& stats);
  void factor();
  void autotune();
};

}  // namespace rb
