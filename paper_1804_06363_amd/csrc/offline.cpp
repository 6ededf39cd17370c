// Offline adaptive greedy sampling (Alg. 4, Sec. 4.2) on the GPU.
//
//   mu_1 = Xi[seed_index]
//   for N = 1..n_max:
//     x(mu_N) = RBCG(A(mu_N), f, W_{N-1})          (BatchSolver, B = 1, FP64; W_0 empty:
//                                                     smoother-only PCG)
//     W_N = orth(W_{N-1}, x(mu_N))                   (classical Gram-Schmidt applied twice
//                                                     with the projection/prolongation
//                                                     kernels; degenerate -> next candidate)
//     A_{N,q}, f_{N,r} grown by one row/column       (eq. 12c)
//     sweep: a(mu) = A_N(mu)^-1 f_N(mu) for all mu   (eq. 12b, batched Cholesky)
//            indicator L1 = sum |a_n|  or  residual ||f - A(mu) W a|| / ||f||
//     mu_{N+1} = argmax over the unpicked candidates (lowest index on ties)
// With use_surrogate the sweep of most steps is replaced by the MLP ranking (mlp.cpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "offline.h"
#include "solver.h"

namespace rb {

GreedyState::GreedyState(rb_ctx* c, const rb_problem* p, const rb_greedy_opts& o, int64_t M_,
                         const double* theta, const double* phi)
    : ctx(c), prob(p), opt(o), M((int)M_) {
  const int Q = p->g.Q, R = p->R;
  hipStream_t st = ctx->stream;
  theta_h.assign(theta, theta + (size_t)M * Q);
  if (phi) phi_h.assign(phi, phi + (size_t)M * R);
  theta_d.alloc(sizeof(double) * (size_t)M * Q);
  RB_HIP(hipMemcpyAsync(theta_d.p, theta, theta_d.bytes, hipMemcpyHostToDevice, st));
  if (phi) {
    phi_d.alloc(sizeof(double) * (size_t)M * R);
    RB_HIP(hipMemcpyAsync(phi_d.p, phi, phi_d.bytes, hipMemcpyHostToDevice, st));
  }
  a_ld = std::max(16, (o.n_max + 15) / 16 * 16);
  // the prolongation reads coefficient rows in groups of 8: pad by 8 zero rows
  coeffs.alloc(sizeof(double) * (size_t)(M + 8) * a_ld);
  ind.alloc(sizeof(double) * (size_t)M);
  l1.alloc(sizeof(double) * (size_t)M);
  cstatus.alloc(sizeof(int) * (size_t)M);
  excluded.alloc(sizeof(int) * (size_t)M);
  amax.alloc(64);
  excl_h.assign(M, 0);
  // the basis grows in place: W64 has room for n_max columns
  bs = std::make_unique<rb_basis>();
  bs->ctx = ctx;
  bs->prob = p;
  bs->n = 0;
  bs->ld = p->ld;
  bs->W64.alloc(sizeof(double) * ((size_t)basis_rows(o.n_max) * p->ld + kBasisTail));
  bs->cap = o.n_max;
  w.alloc(sizeof(double) * p->ld);
  const int ncN = stencil_chunks_all(p->g.N);
  part.alloc(sizeof(double) * (size_t)std::max(ncN, 1) * 8);
  // ||f||^2 of the shared right-hand side (R = 1); scaled by phi^2 per candidate
  const int nc = launch_dot(p->f.as<double>(), p->f.as<double>(), p->ld, p->g.N, 1,
                            part.as<double>(), 4, st);
  std::vector<double> ph(nc);
  RB_HIP(hipMemcpyAsync(ph.data(), part.p, sizeof(double) * nc, hipMemcpyDeviceToHost, st));
  RB_HIP(hipStreamSynchronize(st));
  fnorm2 = 0.0;
  for (double v : ph) fnorm2 += v;
}

void GreedyState::adopt(const rb_basis* src) {
  RB_REQUIRE(src->prob == prob, RB_EINVAL, "basis belongs to another problem");
  RB_REQUIRE(src->n <= opt.n_max, RB_EINVAL, "basis larger than the greedy's capacity");
  hipStream_t st = ctx->stream;
  if (src->n > 0)
    RB_HIP(hipMemcpyAsync(bs->W64.p, src->W64.p, sizeof(double) * (size_t)src->n * prob->ld,
                          hipMemcpyDeviceToDevice, st));
  bs->n = src->n;
  bs->AN_host = src->AN_host;
  bs->fN_host = src->fN_host;
  bs->AN.alloc(sizeof(double) * std::max<size_t>(1, bs->AN_host.size()));
  bs->fN.alloc(sizeof(double) * std::max<size_t>(1, bs->fN_host.size()));
  if (!bs->AN_host.empty())
    RB_HIP(hipMemcpyAsync(bs->AN.p, bs->AN_host.data(), sizeof(double) * bs->AN_host.size(),
                          hipMemcpyHostToDevice, st));
  if (!bs->fN_host.empty())
    RB_HIP(hipMemcpyAsync(bs->fN.p, bs->fN_host.data(), sizeof(double) * bs->fN_host.size(),
                          hipMemcpyHostToDevice, st));
  RB_HIP(hipStreamSynchronize(st));
}

double GreedyState::norm(const double* v) {
  hipStream_t st = ctx->stream;
  const int nc = launch_dot(v, v, prob->ld, prob->g.N, 1, part.as<double>(), 4, st);
  std::vector<double> ph(nc);
  RB_HIP(hipMemcpyAsync(ph.data(), part.p, sizeof(double) * nc, hipMemcpyDeviceToHost, st));
  RB_HIP(hipStreamSynchronize(st));
  double s = 0.0;
  for (double x : ph) s += x;
  return std::sqrt(s);
}

// Snapshot solve of Alg. 4: RBCG with the current basis (FP64 CG; the preconditioner in
// opt.snapshot_prec).  Returns its iteration count; the solution (storage order) is left
// in `w`.
int GreedyState::snapshot(int mu) {
  rb_solve_opts so;
  rb_solve_opts_default(&so);
  so.rtol = opt.snapshot_rtol;
  so.maxit = opt.snapshot_maxit;
  so.beta_flexible = opt.snapshot_flexible;
  so.precond_prec = opt.snapshot_prec;
  so.smooth_sweeps = opt.snapshot_sweeps;
  const double* th = theta_h.data() + (size_t)mu * prob->g.Q;
  const double* ph = phi_h.empty() ? nullptr : phi_h.data() + (size_t)mu * prob->R;
  BatchSolver s(ctx, prob, bs.get(), so, 1, th, ph, nullptr);
  s.run();
  std::vector<rb_query_stats> stt;
  s.gather(nullptr, 0, stt);
  RB_REQUIRE(stt[0].status == RB_OK, stt[0].status,
             "snapshot solve failed (status " + std::to_string((int)stt[0].status) + ")");
  RB_HIP(hipMemcpyAsync(w.p, s.x.p, sizeof(double) * prob->ld, hipMemcpyDeviceToDevice,
                        ctx->stream));
  RB_HIP(hipStreamSynchronize(ctx->stream));
  return stt[0].iters;
}

// w <- w - W (W^T w), twice ("twice is enough"); appends w/||w|| as a new column.
// Returns false if the remainder is below 1e-12 ||x|| (snapshot already in span W).
bool GreedyState::orthonormalize_append() {
  hipStream_t st = ctx->stream;
  const rb_problem* p = prob;
  const int n = bs->n;
  const double nx = norm(w.as<double>());
  RB_REQUIRE(nx > 0.0 && std::isfinite(nx), RB_EDEGENERATE, "zero or non-finite snapshot");
  if (n > 0) {
    const ProjPlan pl = plan_projection(p->g.N, 1, n, 2048);
    DevBuf pp(sizeof(double) * (size_t)pl.chunks * pl.nj);
    DevBuf t(sizeof(double) * 8 * 128);  // prolongation reads 8 rows of e
    DevBuf one(sizeof(int));
    launch_fill<int>(one.as<int>(), 0, 1, 1, 1, st);
    for (int pass = 0; pass < 2; ++pass) {
      launch_projection(pl, RB_PREC_FP64, w.as<double>(), p->ld, bs->W64.p, p->ld, n, 1,
                        one.as<int>(), pp.p, st);
      launch_reduce_solve(true, pp.p, pl.chunks, 1, pl.nj, n, nullptr, nullptr, nullptr,
                          t.as<double>(), nullptr, nullptr, 16, false, st);
      launch_scale(t.as<double>(), t.as<double>(), n, -1.0, st);
      launch_prolong(RB_PREC_FP64, bs->W64.p, p->ld, n, t.as<double>(), nullptr, n, 1,
                     one.as<int>(), w.p, true, p->ld, 0, p->g.N, true, st);
    }
  }
  const double nw = norm(w.as<double>());
  if (!(nw >= 1e-12 * nx)) return false;
  launch_scale(bs->W64.as<double>() + (size_t)n * p->ld, w.as<double>(), p->ld, 1.0 / nw, st);
  bs->n = n + 1;  // a reduced-precision copy picks the new column up on its next use
  compute_reduced(bs.get(), n);
  return true;
}

// Sweep of the true indicator over the candidates listed in `idx` (all if empty):
// fills ind[m] for those candidates.
void GreedyState::sweep(const std::vector<int>& idx) {
  hipStream_t st = ctx->stream;
  const rb_problem* p = prob;
  const int n = bs->n, Q = p->g.Q, R = p->R;
  const bool all = idx.empty();
  const int cnt = all ? M : (int)idx.size();
  // gather the parameters of the listed candidates
  const double* th_d = theta_d.as<double>();
  const double* ph_d = phi_d.p ? phi_d.as<double>() : nullptr;
  DevBuf thg, phg;
  if (!all) {
    std::vector<double> th((size_t)cnt * Q), ph;
    for (int k = 0; k < cnt; ++k)
      std::copy(theta_h.begin() + (size_t)idx[k] * Q, theta_h.begin() + (size_t)(idx[k] + 1) * Q,
                th.begin() + (size_t)k * Q);
    thg.alloc(sizeof(double) * th.size());
    RB_HIP(hipMemcpyAsync(thg.p, th.data(), thg.bytes, hipMemcpyHostToDevice, st));
    th_d = thg.as<double>();
    if (!phi_h.empty()) {
      ph.resize((size_t)cnt * R);
      for (int k = 0; k < cnt; ++k)
        std::copy(phi_h.begin() + (size_t)idx[k] * R, phi_h.begin() + (size_t)(idx[k] + 1) * R,
                  ph.begin() + (size_t)k * R);
      phg.alloc(sizeof(double) * ph.size());
      RB_HIP(hipMemcpyAsync(phg.p, ph.data(), phg.bytes, hipMemcpyHostToDevice, st));
      ph_d = phg.as<double>();
    }
  }
  // reduced coefficients and the L1 indicator of every listed candidate
  launch_sweep_coeffs(bs->AN.as<double>(), bs->fN.as<double>(), n, Q, R, cnt, th_d, ph_d,
                      coeffs.as<double>(), a_ld, l1.as<double>(), cstatus.as<int>(), st);
  std::vector<double> vals(cnt);
  if (opt.indicator == RB_IND_L1) {
    RB_HIP(hipMemcpyAsync(vals.data(), l1.p, sizeof(double) * cnt, hipMemcpyDeviceToHost, st));
    RB_HIP(hipStreamSynchronize(st));
  } else {
    // residual indicator ||f - A(mu) W a(mu)|| / ||f||, in chunks of CB candidates
    const int64_t ld = p->ld;
    int CB = (int)std::min<int64_t>(1024, std::max<int64_t>(8, (int64_t)(2ll << 30) / (16 * ld)));
    CB = std::min(CB, cnt);
    DevBuf X(sizeof(double) * (size_t)CB * ld), Rv(sizeof(double) * (size_t)CB * ld);
    DevBuf coef(sizeof(double) * (size_t)CB * p->g.ct_size);
    DevBuf ones(sizeof(int) * CB), sc(sizeof(double) * CB), s2(sizeof(double) * CB);
    const int ncN = stencil_chunks_all(p->g.N);
    DevBuf prt(sizeof(double) * (size_t)CB * ncN);
    launch_fill<int>(ones.as<int>(), 0, CB, 1, 1, st);
    std::vector<double> scale(CB), ss(CB);
    for (int c0 = 0; c0 < cnt; c0 += CB) {
      const int cb = std::min(CB, cnt - c0);
      for (int k = 0; k < cb; ++k) {
        const int m = all ? c0 + k : idx[c0 + k];
        scale[k] = (R == 1 && !phi_h.empty()) ? phi_h[(size_t)m] : 1.0;
      }
      RB_HIP(hipMemcpyAsync(sc.p, scale.data(), sizeof(double) * cb, hipMemcpyHostToDevice, st));
      // x_hat = W a for the chunk (every node)
      launch_prolong(RB_PREC_FP64, bs->W64.p, ld, n, coeffs.as<double>() + (size_t)c0 * a_ld,
                     nullptr, a_ld, cb, ones.as<int>(), X.p, true, ld, 0, p->g.N, false, st);
      launch_coef_tables(p->g, cb, th_d + (size_t)c0 * Q, nullptr, coef.as<double>(), st);
      launch_apply(p->g, ld, cb, coef.as<double>(), X.as<double>(), Rv.as<double>(), 1,
                   p->f.as<double>(), 0, sc.as<double>(), ones.as<int>(), prt.as<double>(), st);
      launch_fin_sum(prt.as<double>(), ncN, ncN, s2.as<double>(), nullptr, cb, st);
      RB_HIP(hipMemcpyAsync(ss.data(), s2.p, sizeof(double) * cb, hipMemcpyDeviceToHost, st));
      RB_HIP(hipStreamSynchronize(st));
      for (int k = 0; k < cb; ++k)
        vals[c0 + k] = std::sqrt(ss[k] / (fnorm2 * scale[k] * scale[k]));
    }
    std::vector<int> cs(cnt);
    RB_HIP(hipMemcpy(cs.data(), cstatus.p, sizeof(int) * cnt, hipMemcpyDeviceToHost));
    for (int k = 0; k < cnt; ++k)
      if (cs[k] != RB_OK) vals[k] = std::nan("");
  }
  if (ind_h.size() != (size_t)M) ind_h.assign(M, -HUGE_VAL);
  for (int k = 0; k < cnt; ++k) ind_h[all ? k : idx[k]] = vals[k];
  true_evals += cnt;
}

// Next sample of Alg. 4 on the device: argmax of ind over the candidates not excluded.
int GreedyState::pick(double* value) {
  hipStream_t st = ctx->stream;
  RB_HIP(hipMemcpyAsync(ind.p, ind_h.data(), sizeof(double) * M, hipMemcpyHostToDevice, st));
  RB_HIP(hipMemcpyAsync(excluded.p, excl_h.data(), sizeof(int) * M, hipMemcpyHostToDevice, st));
  double* ov = amax.as<double>();
  int* oi = (int*)(amax.as<char>() + 8);
  int* on = (int*)(amax.as<char>() + 12);
  launch_argmax(ind.as<double>(), excluded.as<int>(), M, ov, oi, on, st);
  char buf[16];
  RB_HIP(hipMemcpyAsync(buf, amax.p, 16, hipMemcpyDeviceToHost, st));
  RB_HIP(hipStreamSynchronize(st));
  double v;
  int i, nanf;
  std::memcpy(&v, buf, 8);
  std::memcpy(&i, buf + 8, 4);
  std::memcpy(&nanf, buf + 12, 4);
  RB_REQUIRE(!nanf, RB_ENOTSPD, "indicator is NaN for some candidate (reduced matrix not SPD)");
  if (value) *value = v;
  return i;
}

}  // namespace rb

using namespace rb;

extern "C" void rb_greedy_opts_default(rb_greedy_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(rb_greedy_opts);
  o->n_max = 10;
  o->seed_index = 0;
  o->indicator = RB_IND_RESIDUAL;
  o->snapshot_rtol = 1e-10;
  o->snapshot_maxit = 5000;
  o->snapshot_flexible = 1;
  o->use_surrogate = 0;
  o->topk = 256;
  o->explore = 64;
  o->full_sweep_every = 10;
  o->warmup_full_sweeps = 4;
  o->train_steps = 50;
  o->lr = 1e-3;
  o->mu_lo = 0.1;
  o->mu_hi = 10.0;
  o->seed = 1234;
  o->snapshot_prec = RB_PREC_FP64;
  o->surrogate_prec = RB_PREC_BF16;
  o->snapshot_sweeps = 1;
}

extern "C" rb_status rb_offline_build(rb_ctx* ctx, const rb_problem* prob,
                                      const rb_greedy_opts* opts, int64_t M, int P,
                                      const double* mu, const double* theta, const double* phi,
                                      rb_basis** out, rb_greedy_report* rep) {
  try {
    RB_REQUIRE(ctx && prob && opts && theta && out, RB_EINVAL, "null argument");
    RB_REQUIRE(opts->struct_size == sizeof(rb_greedy_opts), RB_EINVAL,
               "rb_greedy_opts.struct_size mismatch");
    RB_REQUIRE(opts->snapshot_prec == RB_PREC_FP64 || opts->snapshot_prec == RB_PREC_FP32,
               RB_EINVAL, "snapshot_prec must be FP64 or FP32");
    RB_REQUIRE(opts->snapshot_sweeps >= 1 && opts->snapshot_sweeps <= 64, RB_EINVAL,
               "snapshot_sweeps must be in 1..64");
    RB_REQUIRE(M >= 1 && M < (1 << 30), RB_EINVAL, "bad training-set size");
    RB_REQUIRE(opts->n_max >= 1 && opts->n_max <= 80, RB_EINVAL, "n_max must be 1..80");
    RB_REQUIRE(opts->seed_index >= 0 && opts->seed_index < M, RB_EINVAL, "bad seed_index");
    RB_REQUIRE(opts->indicator == RB_IND_L1 || opts->indicator == RB_IND_RESIDUAL, RB_EINVAL,
               "bad indicator");
    RB_REQUIRE(opts->indicator == RB_IND_L1 || prob->R == 1, RB_EUNSUPPORTED,
               "residual indicator needs R = 1");
    RB_REQUIRE(!opts->use_surrogate || (mu && P >= 1 && P <= 64), RB_EINVAL,
               "surrogate needs mu with 1 <= P <= 64");
    RB_REQUIRE(opts->surrogate_prec == RB_PREC_BF16 || opts->surrogate_prec == RB_PREC_FP32,
               RB_EINVAL, "surrogate_prec must be BF16 or FP32");
    RB_REQUIRE(opts->topk >= 0 && opts->explore >= 0 && opts->train_steps >= 0, RB_EINVAL,
               "bad surrogate options");
    for (int64_t i = 0; i < M * prob->g.Q; ++i)
      RB_REQUIRE(std::isfinite(theta[i]), RB_EINVAL, "theta contains NaN or Inf");
    const auto t0 = std::chrono::steady_clock::now();
    DeviceGuard dg(ctx->device);
    GreedyState gs(ctx, prob, *opts, M, theta, phi);
    std::unique_ptr<Surrogate> sur;
    if (opts->use_surrogate) sur = std::make_unique<Surrogate>(gs, mu, P);
    std::vector<int64_t> picks;
    std::vector<double> maxind;
    std::vector<int> snap_it;
    int mu_next = (int)opts->seed_index;
    int step = 0;
    while (gs.bs->n < opts->n_max) {
      const int it = gs.snapshot(mu_next);                  // snapshot
      gs.excl_h[mu_next] = 1;
      if (!gs.orthonormalize_append()) {                    // degenerate snapshot
        RB_REQUIRE(!gs.ind_h.empty(), RB_EDEGENERATE, "first snapshot is degenerate");
        mu_next = gs.pick(nullptr);
        RB_REQUIRE(mu_next >= 0, RB_EDEGENERATE, "no candidate left");
        continue;
      }
      picks.push_back(mu_next);
      snap_it.push_back(it);
      gs.bs->picks.push_back(mu_next);
      ++step;
      double v = 0.0;
      int nxt;
      if (sur)
        nxt = sur->step(step, &v);                          // sweep + pick, surrogate
      else {
        gs.sweep({});                                       // indicator sweep
        gs.full_sweeps++;
        nxt = gs.pick(&v);                                  // next sample
      }
      maxind.push_back(v);
      if (nxt < 0) break;
      mu_next = nxt;
    }
    if (rep) {
      rep->n_built = gs.bs->n;
      for (size_t i = 0; i < picks.size() && i < (size_t)opts->n_max; ++i) {
        if (rep->picks) rep->picks[i] = picks[i];
        if (rep->max_indicator) rep->max_indicator[i] = maxind[i];
        if (rep->snapshot_iters) rep->snapshot_iters[i] = snap_it[i];
      }
      rep->true_evals = gs.true_evals;
      rep->full_sweeps = gs.full_sweeps;
      rep->seconds =
          std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      rep->mlp_loss = sur ? sur->last_loss : 0.0;
      rep->surrogate_fallbacks = sur ? sur->fallbacks : 0;
    }
    *out = gs.bs.release();
    return RB_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return RB_EINVAL;
  }
}

// Snapshot solves and basis updates of Alg. 4 for a given parameter sequence (the
// multi-fidelity construction of Sec. 4.2: the parameters are the picks of a greedy on a coarse grid).
extern "C" rb_status rb_basis_from_parameters(rb_ctx* ctx, const rb_problem* prob,
                                              const rb_greedy_opts* opts, int K,
                                              const double* theta, const double* phi,
                                              rb_basis** out, rb_greedy_report* rep) {
  try {
    RB_REQUIRE(ctx && prob && opts && theta && out, RB_EINVAL, "null argument");
    RB_REQUIRE(opts->struct_size == sizeof(rb_greedy_opts), RB_EINVAL,
               "rb_greedy_opts.struct_size mismatch");
    RB_REQUIRE(opts->snapshot_prec == RB_PREC_FP64 || opts->snapshot_prec == RB_PREC_FP32,
               RB_EINVAL, "snapshot_prec must be FP64 or FP32");
    RB_REQUIRE(opts->snapshot_sweeps >= 1 && opts->snapshot_sweeps <= 64, RB_EINVAL,
               "snapshot_sweeps must be in 1..64");
    RB_REQUIRE(K >= 1 && K <= 80, RB_EINVAL, "K must be 1..80");
    for (int64_t i = 0; i < (int64_t)K * prob->g.Q; ++i)
      RB_REQUIRE(std::isfinite(theta[i]), RB_EINVAL, "theta contains NaN or Inf");
    const auto t0 = std::chrono::steady_clock::now();
    DeviceGuard dg(ctx->device);
    rb_greedy_opts o = *opts;
    o.n_max = K;
    o.use_surrogate = 0;
    GreedyState gs(ctx, prob, o, K, theta, phi);
    std::vector<int64_t> used;
    std::vector<int> snap_it;
    for (int i = 0; i < K; ++i) {
      const int it = gs.snapshot(i);            // snapshot
      if (!gs.orthonormalize_append()) continue;  // degenerate: skipped
      used.push_back(i);
      snap_it.push_back(it);
      gs.bs->picks.push_back(i);
    }
    RB_REQUIRE(gs.bs->n > 0, RB_EDEGENERATE, "every snapshot was degenerate");
    if (rep) {
      rep->n_built = gs.bs->n;
      for (size_t i = 0; i < used.size(); ++i) {
        if (rep->picks) rep->picks[i] = used[i];
        if (rep->max_indicator) rep->max_indicator[i] = 0.0;
        if (rep->snapshot_iters) rep->snapshot_iters[i] = snap_it[i];
      }
      rep->true_evals = 0;
      rep->full_sweeps = 0;
      rep->seconds =
          std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      rep->mlp_loss = 0.0;
      rep->surrogate_fallbacks = 0;
    }
    *out = gs.bs.release();
    return RB_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return RB_EINVAL;
  }
}
