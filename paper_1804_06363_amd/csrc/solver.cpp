// Batched online solver: drives the HIP kernels of one iteration of RBCG (Alg. 3),
// RBI (Alg. 2) or plain CG for B queries, with device-side stopping tests and a host
// check of the active queries every few iterations (optionally replaying a captured
// HIP graph of two iterations).
#include "solver.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace rb {

static int64_t align64(int64_t v) { return (v + 63) / 64 * 64; }

BatchSolver::BatchSolver(rb_ctx* c, const rb_problem* p, const rb_basis* b,
                         const rb_solve_opts& o, int B_, const double* theta, const double* phi,
                         const int* n_use, hipStream_t stream, Workspace* ws)
    : ctx(c), prob(p), basis(b), opt(o), B(B_), stream_(stream ? stream : c->stream),
      ws_(ws ? ws : &c->ws) {
  // Host-side set-up only: sizes, tile plan and the workspace views.  Nothing is issued
  // on the stream before prepare(), so a workspace that is too small fails here, before
  // any work.
  const StencilGeom& g = prob->g;
  const int Q = g.Q;
  if (opt.solver == RB_SOLVER_CG) {
    basis = nullptr;
    opt.precond_prec = RB_PREC_FP64;
  }
  n = basis ? basis->n : 0;
  nu_h.assign(B, n);
  adaptive = opt.adapt_gamma > 0.0 && opt.solver == RB_SOLVER_RBCG && n > 0;
  if (adaptive && !n_use) std::fill(nu_h.begin(), nu_h.end(), 1);
  if (n_use && basis)
    for (int i = 0; i < B; ++i) {
      RB_REQUIRE(n_use[i] >= 0, RB_EINVAL, "n_use must be >= 0");
      nu_h[i] = std::min(n_use[i], n);
    }
  theta_h.assign(theta, theta + (size_t)B * Q);
  const int R = prob->R;
  sc_h.assign(B, 1.0);
  if (R == 1 && phi)
    for (int i = 0; i < B; ++i) sc_h[i] = phi[i];
  if (R > 1) {
    phi_h.assign((size_t)B * R, 1.0);
    if (phi) std::copy(phi, phi + (size_t)B * R, phi_h.begin());
  }
  e_ld = std::max(16, (n + 15) / 16 * 16);
  y32 = opt.precond_prec != RB_PREC_FP64 && opt.solver != RB_SOLVER_RBI;
  cN = stencil_chunks_all(g.N);
  pstride = std::max(cN, (g.N + 1023) / 1024);
  // partial sums of the colour sweeps: one segment per colour class, in sweep order
  gsegs.n = g.C;
  int64_t acc = 0;
  for (int c = 0; c < g.C; ++c) {
    gsegs.cnt[c] = stencil_chunks(g.coff[c + 1] - g.coff[c]) + 1;  // at most; each sweep
                                                                // records its own count
    gsegs.off[c] = acc;
    acc += (int64_t)B * gsegs.cnt[c];
  }
  jsegs.n = 1;
  jsegs.cnt[0] = cN;
  jsegs.off[0] = 0;
  const int64_t dot_elems = std::max<int64_t>(acc, (int64_t)B * pstride);
  const int64_t L_ = ld();

  // tile choices: cached by the autotuner for this shape, else the defaults
  {
    auto lg = [](int64_t v) { int k = 0; while ((1ll << (k + 1)) <= v) ++k; return k; };
    std::string arch = ctx->prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    tune_key = arch + "|d" + std::to_string(g.dim) + "|N" + std::to_string(lg(g.N)) + "|B" +
               std::to_string(lg(B)) + "|n" + std::to_string((n + 15) / 16) + "|p" +
               std::to_string((int)opt.precond_prec) + "|s" + std::to_string((int)opt.smoother);
    ctx->tuner.load();
    if (const TuneConfig* c = ctx->tuner.find(tune_key)) tc = *c;
    if (opt.stencil_kind) {
      tc.kind_a = tc.kind_b = std::min(opt.stencil_kind, 2);
      tc.kind_gs = opt.stencil_kind == 4 ? 2 : opt.stencil_kind;
      tc.zn_a = tc.zn_b = tc.np_gs = opt.stencil_kind == 4 ? 4 : 0;
    }
    if (opt.prolong_kind) tc.kind_pro = opt.prolong_kind;
  }
  // projection plan first: for batches it reads residual rows in whole query tiles
  if (n > 0) {
    const int target = tc.proj_target ? tc.proj_target : 4 * ctx->prop.multiProcessorCount;
    plan = plan_projection(g.N, B, n, target);
    plan.padded = !plan.wsplit;
    plan_wave_chunks(plan, B, target, opt.precond_prec);
  }
  // rows of r the batched projection may address: whole query groups (a block of four
  // 16 * qt query tiles, or one such tile in wchunk mode)
  rrows = (n > 0 && plan.padded) ? plan.qgroups * (plan.wchunk ? 16 : 64) * plan.qt : B;

  // workspace views
  theta_d = get_ws(WS_THETA, sizeof(double) * B * Q);
  scale_d = get_ws(WS_SCALE, sizeof(double) * B);
  nuse_d = get_ws(WS_NUSE, sizeof(int) * B);
  ones_d = get_ws(WS_ONES, sizeof(int) * B);
  if (R > 1) {
    phi_d = get_ws(WS_PHI, sizeof(double) * (size_t)B * R);
    fb = get_ws(WS_FB, sizeof(double) * (size_t)B * L_);
  }
  coef = get_ws(WS_COEF, sizeof(double) * B * g.ct_size);
  const size_t vb = sizeof(double) * (size_t)B * L_;
  const size_t vr = sizeof(double) * (size_t)rrows * L_;
  x = get_ws(WS_X, vb);
  r0 = get_ws(WS_R0, vr);
  use_r32 = y32 && opt.residual_copy && opt.solver == RB_SOLVER_RBCG && !g.csr;
  pair_x = opt.paired_x_update && opt.solver != RB_SOLVER_RBI && !g.csr;
  if (use_r32) r32 = get_ws(WS_R32, sizeof(float) * (size_t)rrows * L_);
  if (opt.beta_flexible || opt.smoother == RB_SMOOTH_JACOBI || opt.smoother == RB_SMOOTH_NONE)
    r1 = get_ws(WS_R1, vr);
  if (opt.solver != RB_SOLVER_RBI) {
    xc = get_ws(WS_XC, vb);
    p0 = get_ws(WS_P0, vb);
    p1 = get_ws(WS_P1, vb);
    y = get_ws(WS_Y, (y32 ? sizeof(float) : sizeof(double)) * (size_t)B * L_);
    if (opt.smoother == RB_SMOOTH_JACOBI || opt.smoother == RB_SMOOTH_NONE)
      z = get_ws(WS_Z, (y32 ? sizeof(float) : sizeof(double)) * (size_t)B * L_);
    fused_ok = opt.solver == RB_SOLVER_RBCG && opt.smoother == RB_SMOOTH_RBGS &&
               opt.smooth_sweeps <= 1 && gs_fused_supported(g);
    if (fused_ok) z = get_ws(WS_Z, (y32 ? sizeof(float) : sizeof(double)) * (size_t)B * L_);
  }
  part_m = get_ws(WS_PM, sizeof(double) * (size_t)B * pstride);
  if (opt.floor_factor > 0.0) part_m2 = get_ws(WS_PM2, sizeof(double) * (size_t)B * pstride);
  part_r0 = get_ws(WS_PR0, sizeof(double) * (size_t)dot_elems);
  part_r1 = get_ws(WS_PR1, sizeof(double) * (size_t)dot_elems);
  if (n > 0) {
    const size_t accb = opt.precond_prec == RB_PREC_FP64 ? sizeof(double) : sizeof(float);
    // room for the largest candidate plan of the autotuner
    ProjPlan big = plan_projection(g.N, B, n, 4096);
    big.padded = !big.wsplit;
    plan_wave_chunks(big, B, 4096, opt.precond_prec);
    projpart = get_ws(WS_PROJ, accb * (size_t)std::max(plan.chunks, big.chunks) * B * plan.nj);
    L = get_ws(WS_L, sizeof(double) * (size_t)B * n * n);
    // the prolongations read e in groups of up to 256 queries: padded rows
    const int Bp = padded_queries(B);
    e64 = get_ws(WS_E64, sizeof(double) * (size_t)Bp * e_ld);
    e32 = get_ws(WS_E32, sizeof(float) * (size_t)Bp * e_ld);
    qlist = get_ws(WS_QLIST, sizeof(int) * ((size_t)B + 1));
  }
  qbuf = get_ws(WS_Q, (sizeof(double) * 9 + sizeof(int) * 7) * (size_t)B);
  char* qb = qbuf.as<char>();
  auto takeD = [&](double*& d) { d = (double*)qb; qb += sizeof(double) * B; };
  auto takeI = [&](int*& d) { d = (int*)qb; qb += sizeof(int) * B; };
  takeD(q.fnorm2); takeD(q.rho); takeD(q.alpha); takeD(q.beta); takeD(q.rel_rec);
  takeD(q.rel_true); takeD(q.scalar); takeD(q.rr_in); takeD(q.apend);
  if (!pair_x) q.apend = nullptr;
  takeI(q.active); takeI(q.status); takeI(q.iters); takeI(q.flag); takeI(q.restart);
  takeI(q.at_floor);
  takeI(q.stalls);
  if (adaptive) {
    q.nuse = nuse_d.as<int>();
    q.gamma2 = opt.adapt_gamma * opt.adapt_gamma;
    q.nmax = n;
  }
}

// Uploads the per-query inputs, builds the coefficient tables and the right-hand sides,
// and sets the per-query state; every buffer a solve reads before writing is set here.
void BatchSolver::prepare() {
  const StencilGeom& g = prob->g;
  const int Q = g.Q, R = prob->R;
  const int64_t L_ = ld();
  hipStream_t st = s();
  RB_HIP(hipMemcpyAsync(theta_d.p, theta_h.data(), sizeof(double) * B * Q, hipMemcpyHostToDevice,
                        st));
  RB_HIP(hipMemcpyAsync(nuse_d.p, nu_h.data(), sizeof(int) * B, hipMemcpyHostToDevice, st));
  launch_fill<int>(ones_d.as<int>(), 0, B, 1, 1, st);
  if (R == 1) {
    f_base = prob->f.as<double>();
    f_ld = 0;
  } else {
    // f_b = sum_r phi_br f_r, formed on the device from the terms in storage order
    RB_HIP(hipMemcpyAsync(phi_d.p, phi_h.data(), sizeof(double) * (size_t)B * R,
                          hipMemcpyHostToDevice, st));
    launch_combine_rhs(prob->f.as<double>(), L_, R, phi_d.as<double>(), B, g.N, fb.as<double>(),
                       st);
    f_base = fb.as<double>();
    f_ld = L_;
    std::fill(sc_h.begin(), sc_h.end(), 1.0);
  }
  RB_HIP(hipMemcpyAsync(scale_d.p, sc_h.data(), sizeof(double) * B, hipMemcpyHostToDevice, st));
  launch_coef_tables(g, B, theta_d.as<double>(), nullptr, coef.as<double>(), st);
  if (n > 0) {
    Wsh = const_cast<rb_basis*>(basis)->shadow(opt.precond_prec, st);
    const int Bp = padded_queries(B);
    launch_fill<double>(e64.as<double>(), 0, (int64_t)Bp * e_ld, 1, 0.0, st);
    launch_fill<float>(e32.as<float>(), 0, (int64_t)Bp * e_ld, 1, 0.f, st);
  }
  launch_fill<double>(q.fnorm2, 0, 9 * (int64_t)B, 1, 0.0, st);  // through apend
  launch_fill<int>(q.at_floor, 0, (int64_t)B, 1, 0, st);
  launch_fill<int>(q.stalls, 0, (int64_t)B, 1, 0, st);
  launch_fill<int>(q.status, 0, (int64_t)B, 1, (int)RB_OK, st);
  launch_fill<int>(q.active, 0, (int64_t)B, 1, 1, st);
  launch_fill<int>(q.iters, 0, 3 * (int64_t)B, 1, 0, st);  // iters, flag, restart
}

BatchSolver::~BatchSolver() {
  if (graph) (void)hipGraphExecDestroy(graph);
  for (int i = 0; i < 2; ++i) {
    if (hev_[i]) (void)hipEventDestroy(hev_[i]);
    if (hflags_[i]) (void)hipHostFree(hflags_[i]);
  }
}

// Reduced assembly + Cholesky of every query (eq. 12b, Sec. 2.1).  A query whose
// reduced matrix is not SPD is retired with RB_ENOTSPD.
void BatchSolver::factor() {
  if (n == 0) return;
  // adaptive size: factor the whole reduced matrix; the leading n x n block of the
  // factor is the factor of the leading block, so one factorization serves every size
  launch_cholesky(basis->AN.as<double>(), n, prob->g.Q, B, theta_d.as<double>(),
                  adaptive ? nullptr : nuse_d.as<int>(), L.as<double>(), q.status, s());
  // status != OK -> inactive
  std::vector<int> st(B);
  RB_HIP(hipMemcpyAsync(st.data(), q.status, sizeof(int) * B, hipMemcpyDeviceToHost, s()));
  RB_HIP(hipStreamSynchronize(s()));
  std::vector<int> act(B);
  for (int i = 0; i < B; ++i) act[i] = st[i] == RB_OK ? 1 : 0;
  RB_HIP(hipMemcpyAsync(q.active, act.data(), sizeof(int) * B, hipMemcpyHostToDevice, s()));
}

// One application y = RBI(A, r, W, 1) from x = 0, the preconditioner of Alg. 3: one
// iteration of Alg. 2 (coarse correction and smoothing) whose residual is r itself, plus
// the partial sums of y^T r (and y^T r_old).
void BatchSolver::precondition(const double* r, const double* r_old, const float* rc) {
  const StencilGeom& g = prob->g;
  const int64_t L_ = ld();
  hipStream_t st = s();
  const bool flex = opt.beta_flexible && r_old;
  if (opt.solver == RB_SOLVER_CG) {  // identity: y = r
    launch_jacobi<double>(g, B, coef.as<double>(), r, y.as<double>(), L_, 0.0, r, L_,
                          flex ? r_old : nullptr, L_, q.active, part_r0.as<double>(),
                          flex ? part_r1.as<double>() : nullptr, st);
    return;
  }
  const bool full = opt.smoother == RB_SMOOTH_JACOBI || opt.smoother == RB_SMOOTH_NONE;
  const bool fz = fused();
  // coarse correction z = W A_N^-1 W^T r (black nodes only for Gauss-Seidel: the red
  // sweep overwrites every red node and reads only black ones; into z for the fused sweep)
  void* zdst = (full || fz) ? z.p : y.p;
  if (n > 0) {
    // batched path: the projection and the prolongation visit the active queries only
    const int* ql = nullptr;
    if (!plan.wsplit) {
      launch_compact_active(q.active, B, qlist.as<int>(), st);
      ql = qlist.as<int>();
    }
    {
      ProfScope ps(ctx, "project", st);
      launch_projection(plan, opt.precond_prec, r, L_, Wsh, L_, n, B, q.active, projpart.p, st,
                        ql, rc);
    }
    {
      ProfScope ps(ctx, "reduced_solve", st);
      launch_reduce_solve(opt.precond_prec == RB_PREC_FP64, projpart.p, plan.chunks, B, plan.nj,
                          n, nuse_d.as<int>(), L.as<double>(), q.active, nullptr,
                          e64.as<double>(), e32.as<float>(), e_ld, true, st);
    }
    ProfScope ps(ctx, "prolong", st);
    launch_prolong(opt.precond_prec, Wsh, L_, n, e64.as<double>(), e32.as<float>(), e_ld, B,
                   q.active, zdst, !y32, L_, full ? 0 : g.coff[1], g.N, false, st, ql);
  } else {
    const int lo = full ? 0 : g.coff[1];
    if (y32)
      launch_fill<float>((float*)zdst + lo, L_, g.N - lo, B, 0.f, st);
    else
      launch_fill<double>((double*)zdst + lo, L_, g.N - lo, B, 0.0, st);
  }
  double* pr0 = part_r0.as<double>();
  double* pr1 = flex ? part_r1.as<double>() : nullptr;
  if (fz) {  // both colours in one launch; one partial-sum segment
    ProfScope ps(ctx, "gs_fused", st);
    const int cnt =
        y32 ? launch_gs_fused<float>(g, B, coef.as<double>(), z.as<float>(), y.as<float>(), L_, r,
                                     L_, flex ? r_old : nullptr, L_, q.active, pr0, pr1, pstride,
                                     st)
            : launch_gs_fused<double>(g, B, coef.as<double>(), z.as<double>(), y.as<double>(), L_,
                                      r, L_, flex ? r_old : nullptr, L_, q.active, pr0, pr1,
                                      pstride, st);
    RB_REQUIRE(cnt > 0, RB_EUNSUPPORTED, "fused red-black sweep: no tile plan for this grid");
    fsegs.n = 1;
    fsegs.off[0] = 0;
    fsegs.cnt[0] = cnt;
    return;
  }
  // colour class c from the latest values of the others; its y^T r partials go to
  // segment c (only from the sweep that leaves the class final).  Sweeps without dot
  // products read the FP32 copy of r when there is one (y is FP32 then).
  auto sweep = [&](int color, bool dots) {
    ProfScope ps(ctx, color == 0 ? "gs_red" : "gs_black", st);
    if (!dots && rc && y32) {
      launch_gs_color<float, float>(g, color, B, coef.as<double>(), y.as<float>(), L_, rc, L_,
                                    nullptr, nullptr, 0, q.active, nullptr, nullptr, st);
      return;
    }
    double* d0 = dots ? pr0 + gsegs.off[color] : nullptr;
    double* d1 = dots && pr1 ? pr1 + gsegs.off[color] : nullptr;
    // the sweep reports how many partial sums per query it wrote (chunked or marching)
    const int cnt =
        y32 ? launch_gs_color<float>(g, color, B, coef.as<double>(), y.as<float>(), L_, r, L_,
                                     nullptr, flex ? r_old : nullptr, L_, q.active, d0, d1, st)
            : launch_gs_color<double>(g, color, B, coef.as<double>(), y.as<double>(), L_, r, L_,
                                      nullptr, flex ? r_old : nullptr, L_, q.active, d0, d1, st);
    if (dots) gsegs.cnt[color] = cnt;
  };
  const int reps = std::max(1, opt.smooth_sweeps);
  switch (opt.smoother) {
    case RB_SMOOTH_RBGS:
      for (int it = 0; it < reps; ++it)
        for (int c = 0; c < g.C; ++c) sweep(c, it == reps - 1);
      break;
    case RB_SMOOTH_RBGS_SYM:  // forward (classes 0..C-1) then backward (C-1..0); the
      // repeated sweep of class C-1 changes nothing and is skipped
      for (int it = 0; it < reps; ++it) {
        const bool last = it == reps - 1;
        for (int c = 0; c < g.C; ++c) sweep(c, last && c == g.C - 1);
        for (int c = g.C - 2; c >= 0; --c) sweep(c, last);
      }
      break;
    default: {  // Jacobi (omega 2/3) or none (omega 0): y = z + omega D^-1 (r - A z)
      const double om = opt.smoother == RB_SMOOTH_JACOBI ? 2.0 / 3.0 : 0.0;
      if (y32)
        launch_jacobi<float>(g, B, coef.as<double>(), z.as<float>(), y.as<float>(), L_, om, r, L_,
                             flex ? r_old : nullptr, L_, q.active, pr0, pr1, st);
      else
        launch_jacobi<double>(g, B, coef.as<double>(), z.as<double>(), y.as<double>(), L_, om, r,
                              L_, flex ? r_old : nullptr, L_, q.active, pr0, pr1, st);
    }
  }
}

// the partial-sum segments of y^T r for this solve's smoother
const Segs& BatchSolver::dot_segs() const {
  if (opt.solver != RB_SOLVER_CG && fused()) return fsegs;
  const bool gs = opt.solver != RB_SOLVER_CG &&
                  (opt.smoother == RB_SMOOTH_RBGS || opt.smoother == RB_SMOOTH_RBGS_SYM);
  return gs ? gsegs : jsegs;
}

// RBCG start (Alg. 3): x = 0, r = f, y = RBI(A, r, W, 1), p = y (beta = 0).
void BatchSolver::init_cg() {
  const StencilGeom& g = prob->g;
  const int64_t L_ = ld();
  hipStream_t st = s();
  launch_fill<double>(x.as<double>(), L_, L_, B, 0.0, st);
  launch_fill<double>(xc.as<double>(), L_, L_, B, 0.0, st);
  launch_fill<double>(p0.as<double>(), L_, L_, B, 0.0, st);
  launch_fill<double>(p1.as<double>(), L_, L_, B, 0.0, st);
  launch_fill<double>(r0.as<double>(), L_, L_, rrows, 0.0, st);  // also zeroes the padding
  if (r1.p) launch_fill<double>(r1.as<double>(), L_, L_, rrows, 0.0, st);
  float* rc = use_r32 ? r32.as<float>() : nullptr;
  if (rc) launch_fill<float>(rc, L_, L_, rrows, 0.f, st);
  const int ci = launch_init_rhs(f_base, f_ld, scale_d.as<double>(), g.N, r0.as<double>(), L_,
                                 B, part_m.as<double>(), pt, st, rc);
  launch_fin_sum(part_m.as<double>(), ci, ci, q.fnorm2, nullptr, B, st);
  if (adaptive)  // r_0 = f is preconditioned first
    RB_HIP(hipMemcpyAsync(q.rr_in, q.fnorm2, sizeof(double) * B, hipMemcpyDeviceToDevice, st));
  factor();
  launch_fill<int>(q.restart, 0, B, 1, 1, st);
  precondition(r0.as<double>(), nullptr, rc);
  launch_fin_beta(part_r0.as<double>(), nullptr, dot_segs(), q, B, false, st);
}

// One RBCG iteration (Alg. 3) for every active query.
void BatchSolver::iterate_cg(int k) {
  const StencilGeom& g = prob->g;
  const int64_t L_ = ld();
  hipStream_t st = s();
  double* pold = (k & 1) ? p1.as<double>() : p0.as<double>();
  double* pnew = (k & 1) ? p0.as<double>() : p1.as<double>();
  const bool flex = opt.beta_flexible != 0;
  double* rin = (flex && (k & 1)) ? r1.as<double>() : r0.as<double>();
  double* rout = flex ? ((k & 1) ? r0.as<double>() : r1.as<double>()) : rin;
  float* rc = use_r32 ? r32.as<float>() : nullptr;  // FP32 copy of rout
  // the previous iteration's direction update fused with the product: p = y + beta p; A p
  int ca, cb;
  {
    ProfScope ps(ctx, "pass_a", st);
    if (y32)
      ca = launch_pass_a<float>(g, L_, B, coef.as<double>(), y.as<float>(), L_, pold, pnew,
                                q.beta, q.active, part_m.as<double>(), st);
    else
      ca = launch_pass_a<double>(g, L_, B, coef.as<double>(), y.as<double>(), L_, pold, pnew,
                                 q.beta, q.active, part_m.as<double>(), st);
  }
  launch_fin_alpha(part_m.as<double>(), cN, ca, q, B, st);
  // x += alpha p (into the correction xc), r -= alpha A p.  Paired updates: an even
  // iteration leaves its x update to the next one, whose pass B reads and writes x once
  // for both, (x + alpha_k p_k) + alpha_k+1 p_k+1, the same operations in the same order;
  // the pending alpha sits in q.apend and its direction in p1 (the new direction of every
  // even iteration), which a fold before the next pass B applies instead.
  const bool defer = pair_x && !(k & 1);
  {
    ProfScope ps(ctx, "pass_b", st);
    cb = launch_pass_b(g, L_, B, coef.as<double>(), pnew, xc.as<double>(), rin, rout, q.alpha,
                       q.active, part_m.as<double>(), st, rc, !pair_x ? 0 : defer ? 1 : 2,
                       pold, q.apend);
  }
  // stopping test: recursive, then the true residual of the flagged queries, formed from x
  // after the correction accumulated since the previous check is folded into it.  The
  // iterate is x + xc either way; keeping the updates apart from x until a check makes
  // their rounding errors relative to the small correction rather than to x, so a
  // residual replacement is not undone by the rounding of the next cycle's updates
  // (group-wise updating, van der Vorst and Ye 2000).
  const bool fixed = opt.fixed_iters > 0;
  launch_fin_rr(part_m.as<double>(), cN, cb, q, B, opt.rtol, opt.maxit, fixed, st, defer);
  if (!fixed) {
    launch_fold(q.flag, B, x.as<double>(), xc.as<double>(), L_, st, q.apend, p1.as<double>());
    ProfScope ps(ctx, "true_residual", st);
    double* p2 = opt.floor_factor > 0.0 ? part_m2.as<double>() : nullptr;
    launch_apply(g, L_, B, coef.as<double>(), x.as<double>(), rout, 1, f_base, f_ld,
                 scale_d.as<double>(), q.flag, part_m.as<double>(), st, p2, rc);
    launch_fin_true(part_m.as<double>(), cN, cN, q, B, opt.rtol, opt.maxit, st, p2,
                    opt.floor_factor);
  }
  // preconditioning and the new direction coefficient
  precondition(rout, flex ? rin : nullptr, rc);
  launch_fin_beta(part_r0.as<double>(), flex ? part_r1.as<double>() : nullptr, dot_segs(), q, B,
                  flex, st);
}

// ---- stand-alone RBI (Alg. 2) ----------------------------------------------------------
__global__ void k_fin_rbi(QState q, double rtol, int maxit, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B || !q.active[b]) return;
  const double rel = sqrt(q.scalar[b] / q.fnorm2[b]);
  q.rel_true[b] = rel;
  q.rel_rec[b] = rel;
  if (rel <= rtol) {
    q.active[b] = 0;
    q.status[b] = RB_OK;
  } else if (!(rel == rel)) {
    q.active[b] = 0;
    q.status[b] = RB_EBREAKDOWN;
  } else if (q.iters[b] >= maxit) {
    q.active[b] = 0;
    q.status[b] = RB_ENOCONV;
  } else {
    q.iters[b] += 1;
  }
}

void BatchSolver::init_rbi() {
  const StencilGeom& g = prob->g;
  const int64_t L_ = ld();
  hipStream_t st = s();
  launch_fill<double>(x.as<double>(), L_, L_, B, 0.0, st);
  launch_fill<double>(r0.as<double>(), L_, L_, rrows, 0.0, st);
  if (r1.p) launch_fill<double>(r1.as<double>(), L_, L_, rrows, 0.0, st);
  const int ci = launch_init_rhs(f_base, f_ld, scale_d.as<double>(), g.N, r0.as<double>(), L_,
                                 B, part_m.as<double>(), pt, st);
  launch_fin_sum(part_m.as<double>(), ci, ci, q.fnorm2, nullptr, B, st);
  factor();
}

// One iteration of Alg. 2 for every active query (x lives in x, r in r0).
void BatchSolver::iterate_rbi(int k) {
  const StencilGeom& g = prob->g;
  const int64_t L_ = ld();
  hipStream_t st = s();
  double* xc = x.as<double>();
  // r = f - A x, ||r||^2  (the active flags select the queries)
  launch_apply(g, L_, B, coef.as<double>(), xc, r0.as<double>(), 1, f_base, f_ld,
               scale_d.as<double>(), q.active, part_m.as<double>(), st);
  launch_fin_sum(part_m.as<double>(), cN, cN, q.scalar, q.active, B, st);
  // stopping test
  const bool fixed = opt.fixed_iters > 0;
  hipLaunchKernelGGL(k_fin_rbi, dim3((B + 63) / 64), dim3(64), 0, st, q, fixed ? -1.0 : opt.rtol,
                     fixed ? (1 << 30) : opt.maxit, B);
  const bool full = opt.smoother == RB_SMOOTH_JACOBI || opt.smoother == RB_SMOOTH_NONE;
  // coarse correction: x += W A_N^-1 W^T r (black nodes only before a Gauss-Seidel sweep)
  if (n > 0) {
    launch_projection(plan, opt.precond_prec, r0.as<double>(), L_, Wsh, L_, n, B, q.active,
                      projpart.p, st);
    launch_reduce_solve(opt.precond_prec == RB_PREC_FP64, projpart.p, plan.chunks, B, plan.nj, n,
                        nuse_d.as<int>(), L.as<double>(), q.active, nullptr, e64.as<double>(),
                        e32.as<float>(), e_ld, true, st);
    launch_prolong(opt.precond_prec, Wsh, L_, n, e64.as<double>(), e32.as<float>(), e_ld, B,
                   q.active, xc, true, L_, full ? 0 : g.coff[1], g.N, true, st);
  }
  // smoothing: x = S(A, f, x)
  auto sweep = [&](int color) {
    launch_gs_color<double>(g, color, B, coef.as<double>(), xc, L_, f_base, f_ld,
                            scale_d.as<double>(), nullptr, 0, q.active, nullptr, nullptr, st);
  };
  const int reps = std::max(1, opt.smooth_sweeps);
  switch (opt.smoother) {
    case RB_SMOOTH_RBGS:
      for (int it = 0; it < reps; ++it)
        for (int c = 0; c < g.C; ++c) sweep(c);
      break;
    case RB_SMOOTH_RBGS_SYM:
      for (int it = 0; it < reps; ++it) {
        for (int c = 0; c < g.C; ++c) sweep(c);
        for (int c = g.C - 2; c >= 0; --c) sweep(c);
      }
      break;
    case RB_SMOOTH_JACOBI:
      RB_REQUIRE(f_ld == L_ || prob->R == 1, RB_EUNSUPPORTED, "Jacobi RBI");
      // x_new = x + omega D^-1 (f - A x) into r1, copied back into x
      launch_jacobi<double>(g, B, coef.as<double>(), xc, r1.as<double>(), L_, 2.0 / 3.0, f_base,
                            f_ld, nullptr, 0, q.active, nullptr, nullptr, st);
      RB_HIP(hipMemcpyAsync(xc, r1.p, sizeof(double) * (size_t)B * L_, hipMemcpyDeviceToDevice,
                            st));
      break;
    default:
      break;
  }
  (void)k;
}

// Final FP64 true residual of every query (reported in the stats).
void BatchSolver::final_true_residual() {
  const StencilGeom& g = prob->g;
  const int64_t L_ = ld();
  hipStream_t st = s();
  // with paired updates, the last even iteration's of the queries still running, and of
  // those that stopped after one (maxit, breakdown), is still pending
  if (xc.p) launch_fold(nullptr, B, x.as<double>(), xc.as<double>(), L_, st, q.apend,
                        p1.as<double>());
  if (q.apend) launch_fill<double>(q.apend, 0, B, 1, 0.0, st);
  double* tmp = r0.as<double>();
  launch_apply(g, L_, B, coef.as<double>(), x.as<double>(), tmp, 1, f_base, f_ld,
               scale_d.as<double>(), ones_d.as<int>(), part_m.as<double>(), st);
  launch_fin_sum(part_m.as<double>(), cN, cN, q.scalar, nullptr, B, st);
  RB_HIP(hipStreamSynchronize(st));
}

// Times candidate tiles on this solve's own (not yet initialised) buffers and keeps the
// fastest: kind (chunked or z-marching) and queries per block of pass A, pass B and the
// colour sweeps, and the number of projection blocks (timed
// with the reduction of their partials).  Runs before init, so the values it computes
// are overwritten.
void BatchSolver::autotune() {
  if (!opt.autotune || ctx->tuner.find(tune_key) || opt.solver == RB_SOLVER_RBI ||
      opt.stencil_kind || prob->g.csr)
    return;
  const StencilGeom& g = prob->g;
  const int64_t L_ = ld();
  hipStream_t st = s();
  hipEvent_t e0, e1;
  RB_HIP(hipEventCreate(&e0));
  RB_HIP(hipEventCreate(&e1));
  auto timed = [&](auto&& launch) {
    launch();  // warm
    float best = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      RB_HIP(hipEventRecord(e0, st));
      launch();
      RB_HIP(hipEventRecord(e1, st));
      RB_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      RB_HIP(hipEventElapsedTime(&ms, e0, e1));
      best = std::min(best, ms);
    }
    return best;
  };
  const int caps[4] = {1, 2, 4, 8};
  // the kernels as the solve runs them: pass B writing the FP32 copy of r, which the
  // projection and (with several sweeps, most of) the sweeps read
  float* rc = use_r32 ? r32.as<float>() : nullptr;
  const bool gs_copy = rc && y32 && opt.smooth_sweeps > 1;
  TuneConfig best = tc, cur = tc;
  float ta = 1e30f, tb = 1e30f, tg = 1e30f;
  for (int kz : {1, 2, 4}) {  // chunked, z-marching with 2 or 4 nodes per thread (3D only)
    const int kind = kz == 1 ? 1 : 2, zn = kz == 1 ? 0 : kz;
    if (kind == 2 && g.dim != 3) break;
    for (int c : caps) {
      if (c > B || (kind == 2 && c > 4) || (zn == 4 && c > 2)) break;
      // the marching passes with one and (where they fit) two LDS plane buffers
      const int nbs = kind == 2 && zmarch_two_buffers(g, B, c, zn ? zn : 2) ? 2 : 1;
      for (int nb = 1; nb <= nbs; ++nb) {
        cur = best;
        cur.qpb_a = c;
        cur.kind_a = kind;
        cur.zn_a = zn;
        cur.nb_a = nb;
        set_stencil_tiles(cur);
        const float t1 = timed([&] {
          if (y32)
            launch_pass_a<float>(g, L_, B, coef.as<double>(), y.as<float>(), L_,
                                 p0.as<double>(), p1.as<double>(), q.beta, q.active,
                                 part_m.as<double>(), st);
          else
            launch_pass_a<double>(g, L_, B, coef.as<double>(), y.as<double>(), L_,
                                  p0.as<double>(), p1.as<double>(), q.beta, q.active,
                                  part_m.as<double>(), st);
        });
        if (t1 < ta) {
          ta = t1;
          best.qpb_a = c;
          best.kind_a = kind;
          best.zn_a = zn;
          best.nb_a = nb;
        }
      }
      for (int nb = 1; nb <= nbs; ++nb) {
        cur = best;
        cur.qpb_b = c;
        cur.kind_b = kind;
        cur.zn_b = zn;
        cur.nb_b = nb;
        set_stencil_tiles(cur);
        // with paired x updates, the pass B of an even iteration and that of an odd one
        const float t2 = timed([&] {
          for (int xd : {pair_x ? 1 : 0, pair_x ? 2 : -1})
            if (xd >= 0)
              launch_pass_b(g, L_, B, coef.as<double>(), p1.as<double>(), x.as<double>(),
                            r0.as<double>(), r0.as<double>(), q.alpha, q.active,
                            part_m.as<double>(), st, rc, xd, p0.as<double>(), q.alpha);
        });
        if (t2 < tb) {
          tb = t2;
          best.qpb_b = c;
          best.kind_b = kind;
          best.zn_b = zn;
          best.nb_b = nb;
        }
      }
    }
  }
  for (int kp : {1, 2, 4}) {  // chunked, marching with 2 or 4 column pairs per thread (3D)
    const int kind = kp == 1 ? 1 : 2, np = kp == 1 ? 0 : kp;
    if (kind == 2 && g.dim != 3) break;
    for (int c : caps) {
      if (c > B || (kind == 2 && c > 4) || (np == 4 && c > 2)) break;
      cur = best;
      cur.qpb_gs = c;
      cur.kind_gs = kind;
      cur.np_gs = np;
      set_stencil_tiles(cur);
      const float t3 = timed([&] {
        if (gs_copy)
          launch_gs_color<float, float>(g, 0, B, coef.as<double>(), y.as<float>(), L_, rc, L_,
                                        nullptr, nullptr, 0, q.active, nullptr, nullptr, st);
        else if (y32)
          launch_gs_color<float>(g, 0, B, coef.as<double>(), y.as<float>(), L_, r0.as<double>(),
                                 L_, nullptr, nullptr, L_, q.active, part_r0.as<double>(),
                                 nullptr, st);
        else
          launch_gs_color<double>(g, 0, B, coef.as<double>(), y.as<double>(), L_,
                                  r0.as<double>(), L_, nullptr, nullptr, L_, q.active,
                                  part_r0.as<double>(), nullptr, st);
      });
      if (t3 < tg) { tg = t3; best.qpb_gs = c; best.kind_gs = kind; best.np_gs = np; }
    }
  }
  if (fused_ok) {  // both colours in one launch, against two single-colour sweeps
    for (int c : caps) {
      if (c > B || c > 2) break;
      cur = best;
      cur.qpb_gs = c;
      cur.kind_gs = 3;
      set_stencil_tiles(cur);
      int cnt = 0;
      const float t4 = timed([&] {
        cnt = y32 ? launch_gs_fused<float>(g, B, coef.as<double>(), z.as<float>(), y.as<float>(),
                                           L_, r0.as<double>(), L_, nullptr, L_, q.active,
                                           part_r0.as<double>(), nullptr, pstride, st)
                  : launch_gs_fused<double>(g, B, coef.as<double>(), z.as<double>(),
                                            y.as<double>(), L_, r0.as<double>(), L_, nullptr, L_,
                                            q.active, part_r0.as<double>(), nullptr, pstride, st);
      });
      if (cnt > 0 && t4 < 2.f * tg) { tg = 0.5f * t4; best.qpb_gs = c; best.kind_gs = 3; }
    }
  }
  if (n > 0 && !plan.wsplit) {
    float tp = 1e30f;
    for (int target : {256, 512, 1024, 2048, 4096}) {
      ProjPlan pl = plan_projection(g.N, B, n, target);
      pl.padded = true;
      plan_wave_chunks(pl, B, target, opt.precond_prec);
      if (pl.chunks == 0) continue;
      const float t = timed([&] {
        launch_projection(pl, opt.precond_prec, r0.as<double>(), L_, Wsh, L_, n, B, q.active,
                          projpart.p, st, nullptr, rc);
        // the reduction of the chunk partials grows with the number of chunks
        launch_reduce_solve(opt.precond_prec == RB_PREC_FP64, projpart.p, pl.chunks, B, pl.nj,
                            n, nuse_d.as<int>(), L.as<double>(), q.active, nullptr, nullptr,
                            nullptr, e_ld, false, st);
      });
      if (t < tp) { tp = t; best.proj_target = target; }
    }
    plan = plan_projection(g.N, B, n, best.proj_target);
    plan.padded = true;
    plan_wave_chunks(plan, B, best.proj_target, opt.precond_prec);
  }
  if (n > 0 && B >= 16 && y32 && !opt.prolong_kind) {  // batched prolongation: MFMA tiles
                                                       // or the vector units
    const bool full = opt.smoother == RB_SMOOTH_JACOBI || opt.smoother == RB_SMOOTH_NONE;
    const int lo = full ? 0 : g.coff[1];
    launch_fill<float>(e32.as<float>(), e_ld, e_ld, padded_queries(B), 0.f, st);
    float tk[2] = {1e30f, 1e30f};
    for (int kp = 1; kp <= 2; ++kp) {
      cur = best;
      cur.kind_pro = kp;
      set_stencil_tiles(cur);
      tk[kp - 1] = timed([&] {
        launch_prolong(opt.precond_prec, Wsh, L_, n, e64.as<double>(), e32.as<float>(), e_ld, B,
                       q.active, y.p, false, L_, lo, g.N, false, st, nullptr);
      });
    }
    best.kind_pro = tk[1] < tk[0] ? 2 : 1;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  tc = best;
  set_stencil_tiles(tc);
  ctx->tuner.put(tune_key, tc);
  ctx->tuner.save();
}

void BatchSolver::start() {
  prepare();
  rbi_ = opt.solver == RB_SOLVER_RBI;
  set_stencil_tiles(tc);
  autotune();
  if (rbi_)
    init_rbi();
  else
    init_cg();
  fixed_ = opt.fixed_iters > 0;
  k_ = 0;
  chunk_ = opt.check_every > 0 ? opt.check_every : (prob->g.N >= (1 << 18) ? 4 : 16);
  // A second chunk in flight hides the host's read of the flags behind GPU work, at the
  // price of one chunk of near-empty launches after the last query retires: worth it on
  // large grids (a chunk takes milliseconds), not on small ones where launches dominate.
  depth_ = prob->g.N >= (1 << 18) ? 2 : 1;
  if (opt.use_graph && chunk_ % 2) ++chunk_;
  for (int i = 0; i < 2; ++i) {
    if (!hflags_[i]) RB_HIP(hipHostMalloc((void**)&hflags_[i], sizeof(int) * (size_t)std::max(B, 1)));
    if (!hev_[i]) RB_HIP(hipEventCreateWithFlags(&hev_[i], hipEventDisableTiming));
  }
  issued_ = polled_ = 0;
  // RBI: iteration k checks the residual of the k-th iterate first; maxit + 1 checks
  limit_ = fixed_ ? opt.fixed_iters : (rbi_ ? opt.maxit + 1 : opt.maxit);
}

// Issues up to `iters` iterations (fewer at the limit) on this solver's stream.
void BatchSolver::issue(int iters) {
  hipStream_t st = s();
  set_stencil_tiles(tc);
  int todo = std::min(iters, limit_ - k_);
  if (opt.use_graph && !rbi_ && todo >= 2 && k_ % 2 == 0) {
    if (!graph) {
      hipGraph_t gr;
      RB_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      iterate_cg(0);
      iterate_cg(1);
      RB_HIP(hipStreamEndCapture(st, &gr));
      RB_HIP(hipGraphInstantiate(&graph, gr, nullptr, nullptr, 0));
      RB_HIP(hipGraphDestroy(gr));
    }
    // the graph holds iterations (even, odd); k_ is even here
    while (todo >= 2) {
      RB_HIP(hipGraphLaunch(graph, st));
      k_ += 2;
      todo -= 2;
    }
  }
  for (; todo > 0; --todo, ++k_) {
    if (rbi_)
      iterate_rbi(k_);
    else
      iterate_cg(k_);
  }
  const int slot = issued_ % 2;
  if (!fixed_)
    RB_HIP(hipMemcpyAsync(hflags_[slot], q.active, sizeof(int) * B, hipMemcpyDeviceToHost, st));
  RB_HIP(hipEventRecord(hev_[slot], st));
  kdone_[slot] = k_;
  ++issued_;
}

bool BatchSolver::poll() {
  if (polled_ == issued_) return false;
  const int slot = polled_ % 2;
  RB_HIP(hipEventSynchronize(hev_[slot]));
  ++polled_;
  if (s() == ctx->stream) ctx->prof.resolve();
  if (kdone_[slot] >= limit_) return false;
  if (fixed_) return true;
  for (int i = 0; i < B; ++i)
    if (hflags_[slot][i]) return true;
  return false;
}

void BatchSolver::finish() {
  hipStream_t st = s();
  RB_HIP(hipStreamSynchronize(st));
  if (st == ctx->stream) ctx->prof.resolve();
  set_stencil_tiles(TuneConfig{});
  // queries still active after maxit did not converge
  if (!fixed_) {
    std::vector<int> act(B), stt(B);
    RB_HIP(hipMemcpyAsync(act.data(), q.active, sizeof(int) * B, hipMemcpyDeviceToHost, st));
    RB_HIP(hipMemcpyAsync(stt.data(), q.status, sizeof(int) * B, hipMemcpyDeviceToHost, st));
    RB_HIP(hipStreamSynchronize(st));
    bool changed = false;
    for (int i = 0; i < B; ++i)
      if (act[i]) {
        stt[i] = RB_ENOCONV;
        changed = true;
      }
    if (changed) {
      RB_HIP(hipMemcpyAsync(q.status, stt.data(), sizeof(int) * B, hipMemcpyHostToDevice, st));
      RB_HIP(hipStreamSynchronize(st));
    }
  }
}

void BatchSolver::fill() {
  while (more() && issued_ - polled_ < depth_) issue(chunk_);
}

void BatchSolver::run() {
  start();
  do fill();
  while (poll());
  finish();
}

void BatchSolver::gather(double* x_user, int64_t user_ld, std::vector<rb_query_stats>& stats) {
  hipStream_t st = s();
  final_true_residual();
  if (x_user) launch_from_storage(*prob, B, x.as<double>(), ld(), x_user, user_ld, st);
  std::vector<int> it(B), stt(B), nu(B, n), af(B);
  RB_HIP(hipMemcpyAsync(af.data(), q.at_floor, sizeof(int) * B, hipMemcpyDeviceToHost, st));
  std::vector<double> rr(B), rec(B), fn(B);
  if (n > 0)
    RB_HIP(hipMemcpyAsync(nu.data(), nuse_d.p, sizeof(int) * B, hipMemcpyDeviceToHost, st));
  RB_HIP(hipMemcpyAsync(it.data(), q.iters, sizeof(int) * B, hipMemcpyDeviceToHost, st));
  RB_HIP(hipMemcpyAsync(stt.data(), q.status, sizeof(int) * B, hipMemcpyDeviceToHost, st));
  RB_HIP(hipMemcpyAsync(rr.data(), q.scalar, sizeof(double) * B, hipMemcpyDeviceToHost, st));
  RB_HIP(hipMemcpyAsync(rec.data(), q.rel_rec, sizeof(double) * B, hipMemcpyDeviceToHost, st));
  RB_HIP(hipMemcpyAsync(fn.data(), q.fnorm2, sizeof(double) * B, hipMemcpyDeviceToHost, st));
  RB_HIP(hipStreamSynchronize(st));
  stats.resize(B);
  for (int i = 0; i < B; ++i) {
    stats[i].iters = it[i];
    stats[i].status = (rb_status)stt[i];
    stats[i].rel_res_true = std::sqrt(rr[i] / fn[i]);
    stats[i].rel_res_recursive = rec[i];
    stats[i].n_used = n > 0 ? nu[i] : 0;
    stats[i].at_floor = af[i];
  }
}

}  // namespace rb
