// Surrogate-ranked greedy step and the MLP diagnostics of the C ABI.
//
// Protocol of one greedy step N with the surrogate (the true indicator of Alg. 4 still
// decides every pick):
//  - full sweep of the true indicator for the first `warmup_full_sweeps` steps and
//    every `full_sweep_every` steps; it also adds every unpicked candidate to the
//    replay buffer as (features(mu), log10 indicator); targets are standardised over
//    the buffer before training;
//  - otherwise: the network ranks all candidates, the true indicator is evaluated on
//    the top `topk` plus `explore` random unpicked candidates, and the pick is the
//    argmax of the TRUE indicator among them; if the Spearman rank correlation of
//    prediction and truth on the explore set is below 0.5 the step falls back to a
//    full sweep;
//  - the replay buffer keeps the pairs of the last two steps (the indicator shrinks as
//    N grows) and `train_steps` Adam steps on minibatches of 256 follow.
// Random numbers: one counter-based SplitMix64 sequence (seed opts.seed); the initial
// weights take its first H P + H H + H values, the exploration and minibatch draws
// continue from there.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "kernels.h"
#include "mlp.h"
#include "offline.h"

namespace rb {

constexpr int kHidden = 128;
constexpr int kMinibatch = 256;

// Glorot-uniform weights from the counter-based generator (order W1, W2, w3, each
// row-major), zero biases.
static std::vector<float> glorot_init(int P, int H, uint64_t seed) {
  std::vector<float> p((size_t)H * P + H * H + 3 * H + 1, 0.f);
  uint64_t ctr = 0;
  auto fill = [&](size_t off, int fo, int fi) {
    const double a = std::sqrt(6.0 / (fi + fo));
    for (int i = 0; i < fo * fi; ++i) p[off + i] = (float)((2.0 * uniform01(seed, ctr++) - 1.0) * a);
  };
  fill(0, H, P);
  fill((size_t)H * P + H, H, H);
  fill((size_t)H * P + 2 * H + (size_t)H * H, 1, H);
  return p;
}

static std::vector<double> ranks(const std::vector<double>& v) {
  std::vector<int> o(v.size());
  std::iota(o.begin(), o.end(), 0);
  std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return v[a] < v[b]; });
  std::vector<double> r(v.size());
  for (size_t i = 0; i < o.size();) {
    size_t j = i;
    while (j + 1 < o.size() && v[o[j + 1]] == v[o[i]]) ++j;
    const double avg = 0.5 * (double)(i + j);
    for (size_t k = i; k <= j; ++k) r[o[k]] = avg;
    i = j + 1;
  }
  return r;
}

static double spearman(const std::vector<double>& a, const std::vector<double>& b) {
  const size_t n = a.size();
  if (n < 3) return 1.0;
  const std::vector<double> ra = ranks(a), rb_ = ranks(b);
  double ma = 0, mb = 0;
  for (size_t i = 0; i < n; ++i) { ma += ra[i]; mb += rb_[i]; }
  ma /= n; mb /= n;
  double sab = 0, saa = 0, sbb = 0;
  for (size_t i = 0; i < n; ++i) {
    sab += (ra[i] - ma) * (rb_[i] - mb);
    saa += (ra[i] - ma) * (ra[i] - ma);
    sbb += (rb_[i] - mb) * (rb_[i] - mb);
  }
  return (saa > 0 && sbb > 0) ? sab / std::sqrt(saa * sbb) : 0.0;
}

struct Surrogate::Impl {
  MLP net;
  DevBuf U, topk_out, topk_cnt, Xb, Yb, idx_d;
  struct Entry {
    int m;
    float target;
    int step;
  };
  std::vector<Entry> buf;
  uint64_t seed, ctr;
  Impl(int P, int M, bool bf16, hipStream_t st, uint64_t s)
      : net(P, kHidden, bf16, std::max(M, kMinibatch), st), seed(s),
        ctr((uint64_t)kHidden * P + (uint64_t)kHidden * kHidden + kHidden) {}
};

Surrogate::Surrogate(GreedyState& g, const double* mu, int P_) : gs(g), P(P_) {
  hipStream_t st = gs.ctx->stream;
  const int M = gs.M;
  impl = std::make_unique<Impl>(P, M, gs.opt.surrogate_prec != RB_PREC_FP32, st, gs.opt.seed);
  RB_REQUIRE(gs.opt.mu_lo > 0 && gs.opt.mu_hi > gs.opt.mu_lo, RB_EINVAL, "bad mu range");
  const double l0 = std::log10(gs.opt.mu_lo), l1 = std::log10(gs.opt.mu_hi);
  DevBuf mud(sizeof(double) * (size_t)M * P);
  RB_HIP(hipMemcpyAsync(mud.p, mu, mud.bytes, hipMemcpyHostToDevice, st));
  impl->U.alloc(sizeof(float) * (size_t)M * P);
  launch_features(mud.as<double>(), M * P, 0.5 * (l0 + l1), 0.5 * (l1 - l0), impl->U.as<float>(),
                  st);
  const std::vector<float> p0 = glorot_init(P, kHidden, gs.opt.seed);
  impl->net.set_params(p0.data());
  impl->topk_out.alloc(sizeof(int) * (size_t)M);
  impl->topk_cnt.alloc(sizeof(int) * 4);
  impl->Xb.alloc(sizeof(float) * kMinibatch * P);
  impl->Yb.alloc(sizeof(float) * kMinibatch);
  impl->idx_d.alloc(sizeof(int) * kMinibatch);
  RB_HIP(hipStreamSynchronize(st));
}
Surrogate::~Surrogate() = default;

void Surrogate::set_state(const float* params, int nbuf, const int32_t* idx, const float* target,
                          const int32_t* step, uint64_t counter) {
  impl->net.set_params(params);
  impl->buf.clear();
  for (int i = 0; i < nbuf; ++i) {
    RB_REQUIRE(idx[i] >= 0 && idx[i] < gs.M && std::isfinite(target[i]), RB_EINVAL,
               "bad replay-buffer entry");
    impl->buf.push_back({idx[i], target[i], step[i]});
  }
  impl->ctr = counter;
  RB_HIP(hipStreamSynchronize(gs.ctx->stream));
}
void Surrogate::get_params(float* params) { impl->net.get_params(params); }
uint64_t Surrogate::counter() const { return impl->ctr; }
int Surrogate::param_count() const { return impl->net.count; }

int Surrogate::step(int k, double* value) {
  Impl& im = *impl;
  hipStream_t st = gs.ctx->stream;
  const int M = gs.M;
  const rb_greedy_opts& o = gs.opt;
  bool full = k <= o.warmup_full_sweeps || (o.full_sweep_every > 0 && k % o.full_sweep_every == 0);
  last_topk.clear();
  last_explore.clear();
  last_fallback = false;
  std::vector<int> eval;
  int pick = -1;
  double v = 0.0;
  if (!full) {
    // rank every candidate with the network; top-K among the unpicked ones
    im.net.forward(im.U.as<float>(), M);
    RB_HIP(hipMemcpyAsync(gs.excluded.p, gs.excl_h.data(), sizeof(int) * M, hipMemcpyHostToDevice,
                          st));
    launch_topk(im.net.out.as<float>(), gs.excluded.as<int>(), M, o.topk, im.topk_out.as<int>(),
                im.topk_cnt.as<int>(), st);
    int cnt = 0;
    RB_HIP(hipMemcpyAsync(&cnt, im.topk_cnt.p, sizeof(int), hipMemcpyDeviceToHost, st));
    std::vector<float> pred(M);
    RB_HIP(hipMemcpyAsync(pred.data(), im.net.out.p, sizeof(float) * M, hipMemcpyDeviceToHost, st));
    RB_HIP(hipStreamSynchronize(st));
    eval.resize(cnt);
    if (cnt) RB_HIP(hipMemcpy(eval.data(), im.topk_out.p, sizeof(int) * cnt, hipMemcpyDeviceToHost));
    std::sort(eval.begin(), eval.end());  // the top-K set in increasing index order
    last_topk = eval;
    std::vector<char> in(M, 0);
    for (int m : eval) in[m] = 1;
    // exploration: uniformly random unpicked candidates outside the top-K
    std::vector<int> expl;
    for (int tries = 0; (int)expl.size() < o.explore && tries < 100 * std::max(o.explore, 1);
         ++tries) {
      const int m = std::min(M - 1, (int)(uniform01(im.seed, im.ctr++) * M));
      if (gs.excl_h[m] || in[m]) continue;
      in[m] = 1;
      expl.push_back(m);
    }
    last_explore = expl;
    eval.insert(eval.end(), expl.begin(), expl.end());
    if (eval.empty()) {
      last_full = false;
      return -1;
    }
    gs.sweep(eval);  // true indicator on the short list
    // reliability of the ranking on the exploration sample
    std::vector<double> pe, te;
    for (int m : expl) {
      pe.push_back(pred[m]);
      te.push_back(std::log10(std::max(gs.ind_h[m], 1e-300)));
    }
    if ((int)expl.size() >= 3 && spearman(pe, te) < 0.5) {
      full = true;
      last_fallback = true;
      ++fallbacks;
    } else {
      // the pick: argmax of the true indicator among the evaluated candidates
      std::vector<double> keep(M, -HUGE_VAL);
      for (int m : eval) keep[m] = gs.ind_h[m];
      gs.ind_h = keep;
      pick = gs.pick(&v);
    }
  }
  last_full = full;
  if (full) {
    gs.sweep({});
    gs.full_sweeps++;
    pick = gs.pick(&v);
    eval.clear();
    for (int m = 0; m < M; ++m)
      if (!gs.excl_h[m]) eval.push_back(m);
  }
  // replay buffer: pairs of the last two steps, picked candidates dropped
  for (int m : eval)
    if (!gs.excl_h[m] && gs.ind_h[m] > 0 && std::isfinite(gs.ind_h[m]))
      im.buf.push_back({m, (float)std::log10(gs.ind_h[m]), k});
  im.buf.erase(std::remove_if(im.buf.begin(), im.buf.end(),
                              [&](const Impl::Entry& e) { return e.step < k - 1 || gs.excl_h[e.m]; }),
               im.buf.end());
  // training
  if (!im.buf.empty()) {
    // targets standardised over the buffer (the ranking is invariant to affine maps)
    double mean = 0.0, var = 0.0;
    for (const auto& e : im.buf) mean += e.target;
    mean /= (double)im.buf.size();
    for (const auto& e : im.buf) var += (e.target - mean) * (e.target - mean);
    const double sd = std::sqrt(var / (double)im.buf.size()) + 1e-6;
    std::vector<int> idx(kMinibatch);
    std::vector<float> y(kMinibatch);
    const int mb = std::min<int>(kMinibatch, (int)im.buf.size());
    for (int s = 0; s < o.train_steps; ++s) {
      for (int i = 0; i < mb; ++i) {
        const size_t e = std::min(im.buf.size() - 1,
                                  (size_t)(uniform01(im.seed, im.ctr++) * (double)im.buf.size()));
        idx[i] = im.buf[e].m;
        y[i] = (float)((im.buf[e].target - mean) / sd);
      }
      RB_HIP(hipMemcpyAsync(im.idx_d.p, idx.data(), sizeof(int) * mb, hipMemcpyHostToDevice, st));
      RB_HIP(hipMemcpyAsync(im.Yb.p, y.data(), sizeof(float) * mb, hipMemcpyHostToDevice, st));
      launch_gather(im.U.as<float>(), nullptr, P, im.idx_d.as<int>(), mb, im.Xb.as<float>(),
                    nullptr, st);
      im.net.backward(im.Xb.as<float>(), im.Yb.as<float>(), mb);
      im.net.adam(o.lr);
    }
    last_loss = im.net.last_loss();
  }
  if (value) *value = v;
  return pick;
}

}  // namespace rb

using namespace rb;

// ---- diagnostics (C ABI) ------------------------------------------------------------------
template <typename F>
static rb_status mlp_guard(F&& f) {
  try {
    f();
    return RB_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return RB_EINVAL;
  }
}

static void check_mlp_args(rb_ctx* ctx, int P, int H, rb_prec prec, const float* params, int m) {
  RB_REQUIRE(ctx && params, RB_EINVAL, "null argument");
  RB_REQUIRE(P >= 1 && P <= 64 && H >= 16 && H <= 512 && H % 16 == 0, RB_EINVAL,
             "need 1 <= P <= 64 and H a multiple of 16 in [16, 512]");
  RB_REQUIRE(prec == RB_PREC_BF16 || prec == RB_PREC_FP32, RB_EINVAL, "prec must be BF16 or FP32");
  RB_REQUIRE(m >= 1 && m <= (1 << 20), RB_EINVAL, "bad row count");
}

extern "C" rb_status rb_mlp_forward(rb_ctx* ctx, int P, int H, rb_prec prec, const float* params,
                                    int m, const float* X, float* out) {
  return mlp_guard([&] {
    check_mlp_args(ctx, P, H, prec, params, m);
    RB_REQUIRE(X && out, RB_EINVAL, "null argument");
    DeviceGuard dg(ctx->device);
    hipStream_t st = ctx->stream;
    MLP net(P, H, prec == RB_PREC_BF16, m, st);
    net.set_params(params);
    DevBuf Xd(sizeof(float) * (size_t)m * P);
    RB_HIP(hipMemcpyAsync(Xd.p, X, Xd.bytes, hipMemcpyHostToDevice, st));
    net.forward(Xd.as<float>(), m);
    RB_HIP(hipMemcpyAsync(out, net.out.p, sizeof(float) * m, hipMemcpyDeviceToHost, st));
    RB_HIP(hipStreamSynchronize(st));
  });
}

extern "C" rb_status rb_mlp_loss_grad(rb_ctx* ctx, int P, int H, rb_prec prec, const float* params,
                                      int m, const float* X, const float* y, float* loss,
                                      float* grad) {
  return mlp_guard([&] {
    check_mlp_args(ctx, P, H, prec, params, m);
    RB_REQUIRE(X && y && loss && grad, RB_EINVAL, "null argument");
    DeviceGuard dg(ctx->device);
    hipStream_t st = ctx->stream;
    MLP net(P, H, prec == RB_PREC_BF16, m, st);
    net.set_params(params);
    DevBuf Xd(sizeof(float) * (size_t)m * P), yd(sizeof(float) * m);
    RB_HIP(hipMemcpyAsync(Xd.p, X, Xd.bytes, hipMemcpyHostToDevice, st));
    RB_HIP(hipMemcpyAsync(yd.p, y, yd.bytes, hipMemcpyHostToDevice, st));
    net.backward(Xd.as<float>(), yd.as<float>(), m);
    RB_HIP(hipMemcpyAsync(grad, net.grads.p, sizeof(float) * net.count, hipMemcpyDeviceToHost, st));
    *loss = net.last_loss();
  });
}

extern "C" rb_status rb_mlp_train(rb_ctx* ctx, int P, int H, rb_prec prec, float* params, int m,
                                  const float* X, const float* y, int steps, double lr,
                                  float* loss) {
  return mlp_guard([&] {
    check_mlp_args(ctx, P, H, prec, params, m);
    RB_REQUIRE(X && y && steps >= 0 && lr > 0, RB_EINVAL, "bad arguments");
    DeviceGuard dg(ctx->device);
    hipStream_t st = ctx->stream;
    MLP net(P, H, prec == RB_PREC_BF16, m, st);
    net.set_params(params);
    DevBuf Xd(sizeof(float) * (size_t)m * P), yd(sizeof(float) * m);
    RB_HIP(hipMemcpyAsync(Xd.p, X, Xd.bytes, hipMemcpyHostToDevice, st));
    RB_HIP(hipMemcpyAsync(yd.p, y, yd.bytes, hipMemcpyHostToDevice, st));
    for (int s = 0; s < steps; ++s) {
      net.backward(Xd.as<float>(), yd.as<float>(), m);
      net.adam(lr);
    }
    net.get_params(params);
    if (loss) {
      net.backward(Xd.as<float>(), yd.as<float>(), m);
      *loss = net.last_loss();
    }
  });
}

extern "C" rb_status rb_surrogate_step(rb_ctx* ctx, const rb_problem* prob, const rb_basis* basis,
                                       const rb_greedy_opts* opts, int64_t M, int P,
                                       const double* mu, const double* theta,
                                       const int32_t* excluded, float* params, int nbuf,
                                       const int32_t* buf_index, const float* buf_target,
                                       const int32_t* buf_step, int32_t* topk, int32_t* explore,
                                       rb_surrogate_io* io) {
  return mlp_guard([&] {
    RB_REQUIRE(ctx && prob && basis && opts && mu && theta && excluded && params && io,
               RB_EINVAL, "null argument");
    RB_REQUIRE(opts->struct_size == sizeof(rb_greedy_opts), RB_EINVAL,
               "rb_greedy_opts.struct_size mismatch");
    RB_REQUIRE(io->struct_size == sizeof(rb_surrogate_io), RB_EINVAL,
               "rb_surrogate_io.struct_size mismatch");
    RB_REQUIRE(basis->prob == prob && basis->n >= 1, RB_EINVAL,
               "need a non-empty basis of this problem");
    RB_REQUIRE(M >= 1 && M < (1 << 30) && P >= 1 && P <= 64, RB_EINVAL, "bad M or P");
    RB_REQUIRE(io->step >= 1, RB_EINVAL, "step must be >= 1");
    RB_REQUIRE(opts->topk >= 0 && opts->explore >= 0 && opts->train_steps >= 0, RB_EINVAL,
               "bad surrogate options");
    RB_REQUIRE((opts->topk == 0 || topk) && (opts->explore == 0 || explore), RB_EINVAL,
               "topk / explore outputs missing");
    RB_REQUIRE(nbuf >= 0 && (nbuf == 0 || (buf_index && buf_target && buf_step)), RB_EINVAL,
               "bad replay buffer");
    RB_REQUIRE(opts->indicator == RB_IND_L1 || prob->R == 1, RB_EUNSUPPORTED,
               "residual indicator needs R = 1");
    RB_REQUIRE(opts->surrogate_prec == RB_PREC_BF16 || opts->surrogate_prec == RB_PREC_FP32,
               RB_EINVAL, "surrogate_prec must be BF16 or FP32");
    RB_REQUIRE(opts->mu_lo > 0 && opts->mu_hi > opts->mu_lo, RB_EINVAL, "bad mu range");
    for (int64_t i = 0; i < M * prob->g.Q; ++i)
      RB_REQUIRE(std::isfinite(theta[i]), RB_EINVAL, "theta contains NaN or Inf");
    DeviceGuard dg(ctx->device);
    rb_greedy_opts o = *opts;
    o.n_max = basis->n;
    o.use_surrogate = 1;
    GreedyState gs(ctx, prob, o, M, theta, nullptr);
    gs.adopt(basis);
    for (int64_t m = 0; m < M; ++m) gs.excl_h[m] = excluded[m] ? 1 : 0;
    Surrogate sur(gs, mu, P);
    sur.set_state(params, nbuf, buf_index, buf_target, buf_step, io->counter);
    double v = 0.0;
    const int pick = sur.step(io->step, &v);
    std::vector<float> out((size_t)sur.param_count());
    sur.get_params(out.data());
    std::copy(out.begin(), out.end(), params);
    std::copy(sur.last_topk.begin(), sur.last_topk.end(), topk);
    std::copy(sur.last_explore.begin(), sur.last_explore.end(), explore);
    io->counter = sur.counter();
    io->full_sweep = sur.last_full ? 1 : 0;
    io->fallback = sur.last_fallback ? 1 : 0;
    io->n_topk = (int)sur.last_topk.size();
    io->n_explore = (int)sur.last_explore.size();
    io->pick = pick;
    io->value = v;
    io->true_evals = gs.true_evals;
    io->loss = sur.last_loss;
  });
}

extern "C" rb_status rb_topk(rb_ctx* ctx, int M, int K, const float* v, const int* excluded,
                             int* out, int* count) {
  return mlp_guard([&] {
    RB_REQUIRE(ctx && v && out && count && M >= 1 && K >= 0, RB_EINVAL, "bad arguments");
    DeviceGuard dg(ctx->device);
    hipStream_t st = ctx->stream;
    DevBuf vd(sizeof(float) * M), ed(sizeof(int) * M), od(sizeof(int) * M), cd(sizeof(int) * 4);
    RB_HIP(hipMemcpyAsync(vd.p, v, vd.bytes, hipMemcpyHostToDevice, st));
    if (excluded) RB_HIP(hipMemcpyAsync(ed.p, excluded, ed.bytes, hipMemcpyHostToDevice, st));
    launch_topk(vd.as<float>(), ed.as<int>(), M, K, od.as<int>(), cd.as<int>(), st);
    RB_HIP(hipMemcpyAsync(count, cd.p, sizeof(int), hipMemcpyDeviceToHost, st));
    RB_HIP(hipStreamSynchronize(st));
    if (*count > 0)
      RB_HIP(hipMemcpy(out, od.p, sizeof(int) * (size_t)*count, hipMemcpyDeviceToHost));
  });
}
