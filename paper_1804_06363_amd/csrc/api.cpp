// C ABI of librb (include/rb.h): contexts, problems, bases, online solves and the
// single-step diagnostics.  Every entry point catches all C++ exceptions and turns
// them into an rb_status plus a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "solver.h"

namespace rb {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

void DevBuf::alloc(size_t n) {
  release();
  if (n == 0) n = 64;
  if (hipMalloc(&p, n) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
    throw Error{RB_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed"};
  }
  bytes = n;
  if (hipMemset(p, 0, n) != hipSuccess) {
    (void)hipFree(p);
    p = nullptr;
    throw Error{RB_EDEVICE, "hipMemset failed"};
  }
}
void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

hipEvent_t Profiler::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  RB_HIP(hipEventCreate(&e));
  return e;
}
void Profiler::resolve() {
  // pairs whose launches are still in flight stay pending (their events are not reused)
  std::vector<Pending> later;
  for (auto& p : pending) {
    float ms = 0.f;
    const hipError_t e = hipEventElapsedTime(&ms, p.a, p.b);
    if (e == hipErrorNotReady) {
      later.push_back(p);
      continue;
    }
    if (e == hipSuccess) {
      auto it = std::find_if(totals.begin(), totals.end(),
                             [&](const auto& t) { return t.first == p.name; });
      if (it == totals.end()) {
        totals.push_back({p.name, Total{}});
        it = totals.end() - 1;
      }
      it->second.ms += ms;
      it->second.launches += 1;
    }
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  pending.swap(later);
}
Profiler::~Profiler() {
  for (auto& p : pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

}  // namespace rb

using namespace rb;

static int64_t align_ld(int64_t N) { return (N + 63) / 64 * 64; }

// The shadow has room for `cap` columns (zero beyond n); columns are converted once,
// when they first exist, so a basis growing in place (the greedy) costs one column each.
// The conversion runs on the consumer's stream; a consumer on another stream (a group
// of rb_solve_multi, another context) waits for the latest conversion's event, so it
// never reads a half-converted shadow.
const void* rb_basis::shadow(rb_prec prec, hipStream_t consumer) {
  if (prec == RB_PREC_FP64) return W64.p;
  const bool f32 = prec == RB_PREC_FP32;
  DevBuf& dst = f32 ? W32 : W16;
  int& done = f32 ? n32 : n16;
  const size_t es = f32 ? sizeof(float) : sizeof(uint16_t);
  if (!dst.p) {
    dst.alloc(es * ((size_t)basis_rows(std::max(cap, n)) * ld + kBasisTail));
    done = 0;
  }
  if (done < n) {
    if (cast_done && cast_stream != consumer)
      RB_HIP(hipStreamWaitEvent(consumer, cast_done, 0));  // earlier columns' writers
    launch_cast(W64.as<double>() + (size_t)done * ld, static_cast<char*>(dst.p) + es * done * ld,
                (int64_t)(n - done) * ld, prec, consumer);
    done = n;
    if (!cast_done) RB_HIP(hipEventCreateWithFlags(&cast_done, hipEventDisableTiming));
    RB_HIP(hipEventRecord(cast_done, consumer));
    cast_stream = consumer;
  } else if (cast_done && cast_stream != consumer) {
    RB_HIP(hipStreamWaitEvent(consumer, cast_done, 0));
  }
  return dst.p;
}

extern "C" {

const char* rb_last_error(void) { return g_err.c_str(); }
const char* rb_version(void) { return "rb 0.1 gfx950"; }

void rb_solve_opts_default(rb_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(rb_solve_opts);
  o->solver = RB_SOLVER_RBCG;
  o->precond_prec = RB_PREC_FP64;
  o->smoother = RB_SMOOTH_RBGS;
  o->rtol = 1e-10;
  o->maxit = 2000;
  o->residual_copy = 1;
  o->paired_x_update = 1;
}

rb_status rb_ctx_create(int device, void* hip_stream, rb_ctx** out) {
  return guarded([&] {
    RB_REQUIRE(out, RB_EINVAL, "out is NULL");
    int count = 0;
    RB_HIP(hipGetDeviceCount(&count));
    RB_REQUIRE(device >= 0 && device < count, RB_EINVAL, "no such device");
    auto c = std::make_unique<rb_ctx>();
    c->device = device;
    DeviceGuard dg(device);
    RB_HIP(hipGetDeviceProperties(&c->prop, device));
    noalloc_attach(device);  // the fixed buffer of the allocation-free entry points
    if (hip_stream) {
      c->stream = (hipStream_t)hip_stream;
    } else {
      RB_HIP(hipStreamCreate(&c->stream));  // blocking stream, default priority
      c->own_stream = true;
    }
    *out = c.release();
  });
}

rb_status rb_ctx_destroy(rb_ctx* ctx) {
  return guarded([&] {
    if (!ctx) return;
    if (ctx->own_stream && ctx->stream) {
      (void)hipStreamSynchronize(ctx->stream);
      (void)hipStreamDestroy(ctx->stream);
    }
    for (hipStream_t st : ctx->group_streams) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
    delete ctx;
  });
}

rb_status rb_profile_enable(rb_ctx* ctx, int on) {
  return guarded([&] {
    RB_REQUIRE(ctx, RB_EINVAL, "null context");
    RB_HIP(hipStreamSynchronize(ctx->stream));
    ctx->prof.resolve();
    ctx->prof.on = on != 0;
  });
}

rb_status rb_profile_reset(rb_ctx* ctx) {
  return guarded([&] {
    RB_REQUIRE(ctx, RB_EINVAL, "null context");
    RB_HIP(hipStreamSynchronize(ctx->stream));
    ctx->prof.resolve();
    ctx->prof.totals.clear();
  });
}

rb_status rb_profile_get(rb_ctx* ctx, int idx, char* name, size_t name_len, double* ms,
                         int64_t* launches) {
  return guarded([&] {
    RB_REQUIRE(ctx, RB_EINVAL, "null context");
    RB_HIP(hipStreamSynchronize(ctx->stream));
    ctx->prof.resolve();
    RB_REQUIRE(idx >= 0 && idx < (int)ctx->prof.totals.size(), RB_EINVAL, "no such entry");
    const auto& t = ctx->prof.totals[idx];
    if (name && name_len) {
      std::strncpy(name, t.first.c_str(), name_len - 1);
      name[name_len - 1] = 0;
    }
    if (ms) *ms = t.second.ms;
    if (launches) *launches = t.second.launches;
  });
}

rb_status rb_problem_create_stencil(rb_ctx* ctx, const rb_stencil_desc* d, rb_problem** out) {
  return guarded([&] {
    RB_REQUIRE(ctx && d && out, RB_EINVAL, "null argument");
    RB_REQUIRE(d->dim >= 1 && d->dim <= 3, RB_EINVAL, "dim must be 1..3");
    int n[3] = {1, 1, 1}, b[3] = {1, 1, 1};
    int64_t N = 1;
    int Q = 1;
    for (int a = 0; a < d->dim; ++a) {
      n[a] = d->n[a];
      b[a] = d->blocks[a];
      RB_REQUIRE(n[a] >= 1 && b[a] >= 1, RB_EINVAL, "sizes must be positive");
      RB_REQUIRE((n[a] + 1) % b[a] == 0, RB_EINVAL, "(n+1) must be divisible by blocks");
      RB_REQUIRE(b[a] <= 64, RB_EUNSUPPORTED, "at most 64 blocks per axis");
      N *= n[a];
      Q *= b[a];
    }
    RB_REQUIRE(N < (1ll << 30), RB_EUNSUPPORTED, "grid too large (N >= 2^30)");
    RB_REQUIRE(Q <= 64, RB_EUNSUPPORTED, "at most 64 affine terms");
    if (d->dim >= 2) RB_REQUIRE(n[0] % 2 == 1, RB_EUNSUPPORTED, "n[0] must be odd");
    if (d->dim == 3) RB_REQUIRE(n[1] % 2 == 1, RB_EUNSUPPORTED, "n[1] must be odd");
    DeviceGuard dg(ctx->device);
    auto p = std::make_unique<rb_problem>();
    p->ctx = ctx;
    p->desc = *d;
    p->N = N;
    p->ld = align_ld(N);
    StencilGeom& g = p->g;
    g.dim = d->dim;
    g.nx = n[0]; g.ny = n[1]; g.nz = n[2];
    g.bx = b[0]; g.by = b[1]; g.bz = b[2];
    g.Q = Q;
    g.N = (int)N;
    g.NR = (int)((N + 1) / 2);
    g.C = 2;  // red-black
    g.coff[0] = 0;
    g.coff[1] = g.NR;
    g.coff[2] = g.N;
    g.nxy = n[0] * n[1];
    g.div_nx = rbk::make_fastdiv((uint32_t)n[0]);
    g.div_nxy = rbk::make_fastdiv((uint32_t)(n[0] * n[1]));
    // per-axis node tables: state | lo-face block << 8 | hi-face block << 16
    std::vector<uint32_t> tab;
    size_t offs[3];
    for (int a = 0; a < 3; ++a) {
      offs[a] = tab.size();
      const int m = (n[a] + 1) / b[a];
      for (int i = 0; i < n[a]; ++i) {
        const int I = i + 1;
        const int state = (I % m == 0) ? 2 * (I / m) - 1 : 2 * (I / m);
        const int lo = i / m, hi = (i + 1) / m;
        tab.push_back((uint32_t)state | ((uint32_t)lo << 8) | ((uint32_t)hi << 16));
      }
    }
    p->tabs.alloc(sizeof(uint32_t) * tab.size());
    RB_HIP(hipMemcpy(p->tabs.p, tab.data(), sizeof(uint32_t) * tab.size(), hipMemcpyHostToDevice));
    for (int a = 0; a < 3; ++a) g.tab[a] = p->tabs.as<uint32_t>() + offs[a];
    // coefficient tables: axis a -> [normal block][state t1][state t2]
    int off = 0;
    const int S[3] = {2 * b[0] - 1, 2 * b[1] - 1, 2 * b[2] - 1};
    for (int a = 0; a < 3; ++a) {
      const int t1 = a == 0 ? 1 : 0;
      const int t2 = a == 2 ? 1 : 2;
      g.ct_off[a] = off;
      g.ct_s1[a] = S[t1];
      g.ct_s2[a] = S[t2];
      if (a < d->dim) off += b[a] * S[t1] * S[t2];
    }
    g.ct_size = (off + 7) / 8 * 8;
    RB_REQUIRE(g.ct_size <= 1024, RB_EUNSUPPORTED, "too many kappa blocks for the stencil tables");
    // default right-hand side f = 1
    p->R = 1;
    p->f.alloc(sizeof(double) * p->ld);
    launch_fill<double>(p->f.as<double>(), 0, N, 1, 1.0, ctx->stream);
    RB_HIP(hipStreamSynchronize(ctx->stream));
    *out = p.release();
  });
}

rb_status rb_problem_create_csr(rb_ctx* ctx, int64_t N, int Q, const int64_t* rowptr,
                                const int32_t* col, const double* vals, rb_problem** out) {
  return guarded([&] {
    RB_REQUIRE(ctx && rowptr && col && vals && out, RB_EINVAL, "null argument");
    RB_REQUIRE(N >= 1 && Q >= 1, RB_EINVAL, "N and Q must be positive");
    RB_REQUIRE(N < (1ll << 30), RB_EUNSUPPORTED, "N >= 2^30");
    RB_REQUIRE(Q <= 64, RB_EUNSUPPORTED, "at most 64 affine terms");
    RB_REQUIRE(rowptr[0] == 0, RB_EINVAL, "rowptr[0] must be 0");
    for (int64_t i = 0; i < N; ++i)
      RB_REQUIRE(rowptr[i + 1] >= rowptr[i], RB_EINVAL, "rowptr must be non-decreasing");
    const int64_t nnz = rowptr[N];
    RB_REQUIRE(nnz < (1ll << 31), RB_EUNSUPPORTED, "nnz >= 2^31");
    std::vector<int64_t> dpos(N, -1);
    for (int64_t i = 0; i < N; ++i)
      for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        RB_REQUIRE(col[e] >= 0 && col[e] < N, RB_EINVAL, "column index out of range");
        RB_REQUIRE(e == rowptr[i] || col[e] > col[e - 1], RB_EINVAL,
                   "columns must be strictly increasing within a row");
        if (col[e] == i) dpos[i] = e;
      }
    for (int64_t i = 0; i < N; ++i)
      RB_REQUIRE(dpos[i] >= 0, RB_EINVAL, "every row must hold its diagonal");
    check_finite(vals, (size_t)Q * nnz, "vals");
    const int n = (int)N;
    // symmetrised adjacency without the diagonal
    std::vector<int64_t> deg(n + 1, 0);
    for (int i = 0; i < n; ++i)
      for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
        if (col[e] != i) {
          deg[i + 1]++;
          deg[col[e] + 1]++;
        }
    for (int i = 0; i < n; ++i) deg[i + 1] += deg[i];
    std::vector<int> adj(deg[n]);
    {
      std::vector<int64_t> fill(deg.begin(), deg.end() - 1);
      for (int i = 0; i < n; ++i)
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
          if (col[e] != i) {
            adj[fill[i]++] = col[e];
            adj[fill[col[e]]++] = i;
          }
    }
    // first-fit colouring in natural order
    std::vector<int> color(n, -1), stamp(kMaxColors + 1, -1);
    int C = 0;
    for (int i = 0; i < n; ++i) {
      for (int64_t e = deg[i]; e < deg[i + 1]; ++e) {
        const int j = adj[e];
        if (j < i && color[j] <= kMaxColors) stamp[color[j]] = i;
      }
      int c = 0;
      while (c <= kMaxColors && stamp[c] == i) ++c;
      RB_REQUIRE(c < kMaxColors, RB_EUNSUPPORTED, "the colouring needs more than 32 classes");
      color[i] = c;
      C = std::max(C, c + 1);
    }
    DeviceGuard dg(ctx->device);
    auto p = std::make_unique<rb_problem>();
    p->ctx = ctx;
    p->N = N;
    p->ld = align_ld(N);
    StencilGeom& g = p->g;
    g.csr = 1;
    g.dim = 0;
    g.Q = Q;
    g.N = n;
    g.C = C;
    // storage order: colour-major, natural order within a class
    std::vector<int> cnt(C + 1, 0);
    for (int i = 0; i < n; ++i) cnt[color[i] + 1]++;
    for (int c = 0; c < C; ++c) cnt[c + 1] += cnt[c];
    for (int c = 0; c <= C; ++c) g.coff[c] = cnt[c];
    g.NR = g.coff[1];
    p->perm_h.resize(n);
    std::vector<int> inv(n);
    {
      std::vector<int> next(cnt.begin(), cnt.end() - 1);
      for (int i = 0; i < n; ++i) {
        const int pos = next[color[i]]++;
        p->perm_h[pos] = i;
        inv[i] = pos;
      }
    }
    p->color_h = color;
    // sliced ELL: slices of 64 storage rows, width = longest off-diagonal row of the slice
    const int ns = (n + 63) / 64;
    std::vector<int64_t> sptr(ns + 1, 0);
    for (int s = 0; s < ns; ++s) {
      int w = 0;
      for (int pos = 64 * s; pos < std::min(n, 64 * s + 64); ++pos) {
        const int i = p->perm_h[pos];
        w = std::max(w, (int)(rowptr[i + 1] - rowptr[i] - 1));
      }
      sptr[s + 1] = sptr[s] + 64 * (int64_t)w;
    }
    const int64_t total = std::max<int64_t>(sptr[ns], 64);
    std::vector<int> scol(total);
    std::vector<double> sval((size_t)Q * total, 0.0), dg_((size_t)Q * n);
    for (int s = 0; s < ns; ++s) {
      const int w = (int)((sptr[s + 1] - sptr[s]) / 64);
      for (int l = 0; l < 64; ++l) {
        const int pos = 64 * s + l;
        const int i = pos < n ? p->perm_h[pos] : 0;
        int k = 0;
        if (pos < n)
          for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            if (col[e] == i) {
              for (int q = 0; q < Q; ++q) dg_[(size_t)q * n + pos] = vals[(size_t)q * nnz + e];
              continue;
            }
            const int64_t at = sptr[s] + 64 * (int64_t)k + l;
            scol[at] = inv[col[e]];
            for (int q = 0; q < Q; ++q) sval[(size_t)q * total + at] = vals[(size_t)q * nnz + e];
            ++k;
          }
        for (; k < w; ++k) scol[sptr[s] + 64 * (int64_t)k + l] = pos < n ? pos : 0;
      }
    }
    p->sptr.alloc(sizeof(int64_t) * (ns + 1));
    p->scol.alloc(sizeof(int) * total);
    p->sval.alloc(sizeof(double) * (size_t)Q * total);
    p->diag.alloc(sizeof(double) * (size_t)Q * n);
    p->perm.alloc(sizeof(int) * n);
    RB_HIP(hipMemcpy(p->sptr.p, sptr.data(), sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice));
    RB_HIP(hipMemcpy(p->scol.p, scol.data(), sizeof(int) * total, hipMemcpyHostToDevice));
    RB_HIP(hipMemcpy(p->sval.p, sval.data(), sizeof(double) * (size_t)Q * total,
                     hipMemcpyHostToDevice));
    RB_HIP(hipMemcpy(p->diag.p, dg_.data(), sizeof(double) * (size_t)Q * n,
                     hipMemcpyHostToDevice));
    RB_HIP(hipMemcpy(p->perm.p, p->perm_h.data(), sizeof(int) * n, hipMemcpyHostToDevice));
    g.sptr = p->sptr.as<int64_t>();
    g.scol = p->scol.as<int>();
    g.sval = p->sval.as<double>();
    g.sval_ld = total;
    g.diag = p->diag.as<double>();
    g.ct_size = (Q + 7) / 8 * 8;
    p->R = 1;
    p->f.alloc(sizeof(double) * p->ld);
    launch_fill<double>(p->f.as<double>(), 0, N, 1, 1.0, ctx->stream);
    RB_HIP(hipStreamSynchronize(ctx->stream));
    *out = p.release();
  });
}

rb_status rb_problem_colors(const rb_problem* p, int32_t* color, int* ncolors) {
  return guarded([&] {
    RB_REQUIRE(p, RB_EINVAL, "null problem");
    if (ncolors) *ncolors = p->g.C;
    if (color)
      for (int pos = 0; pos < p->g.N; ++pos) {  // class of the storage position's unknown
        int c = 0;
        while (pos >= p->g.coff[c + 1]) ++c;
        color[p->nat_index(pos)] = c;
      }
  });
}

rb_status rb_problem_set_rhs(rb_problem* p, int R, const double* f) {
  return guarded([&] {
    RB_REQUIRE(p && f && R >= 1 && R <= 64, RB_EINVAL, "bad rhs arguments");
    check_finite(f, (size_t)R * p->N, "f");
    DeviceGuard dg(p->ctx->device);
    DevBuf nat(sizeof(double) * (size_t)R * p->N);
    RB_HIP(hipMemcpy(nat.p, f, sizeof(double) * (size_t)R * p->N, hipMemcpyHostToDevice));
    DevBuf sto(sizeof(double) * (size_t)R * p->ld);
    launch_to_storage(*p, R, nat.as<double>(), p->N, sto.as<double>(), p->ld, p->ctx->stream);
    RB_HIP(hipStreamSynchronize(p->ctx->stream));
    p->f = std::move(sto);
    p->R = R;
  });
}

rb_status rb_problem_info(const rb_problem* p, int64_t* N, int* Q, int* R) {
  return guarded([&] {
    RB_REQUIRE(p, RB_EINVAL, "null problem");
    if (N) *N = p->N;
    if (Q) *Q = p->g.Q;
    if (R) *R = p->R;
  });
}

rb_status rb_problem_destroy(rb_problem* p) {
  return guarded([&] { delete p; });
}

}  // extern "C"

namespace rb {

// A_{N,q} = W^T A_q W and f_{N,r} = W^T f_r (eq. 12c) for the columns [j0, n) of the
// basis (rows/columns < j0 are kept), computed with the stencil and projection kernels.
void compute_reduced(rb_basis* bs, int j0) {
  const rb_problem* p = bs->prob;
  const StencilGeom& g = p->g;
  hipStream_t st = bs->ctx->stream;
  const int n = bs->n, Q = g.Q, R = p->R;
  const int nn = n - j0;
  std::vector<double> AN((size_t)Q * n * n, 0.0), fN((size_t)R * n, 0.0);
  for (int q = 0; q < Q; ++q)
    for (int i = 0; i < j0; ++i)
      for (int j = 0; j < j0; ++j)
        AN[((size_t)q * n + i) * n + j] = bs->AN_host[((size_t)q * j0 + i) * j0 + j];
  for (int r = 0; r < R; ++r)
    for (int j = 0; j < j0; ++j) fN[(size_t)r * n + j] = bs->fN_host[(size_t)r * j0 + j];
  if (nn > 0) {
    const int64_t ld = p->ld;
    DevBuf V(sizeof(double) * (size_t)nn * ld);
    DevBuf th(sizeof(double) * (size_t)nn * Q);
    DevBuf coef(sizeof(double) * (size_t)nn * g.ct_size);
    DevBuf t(sizeof(double) * (size_t)nn * n);
    const ProjPlan pl = plan_projection(g.N, nn, n, 2048);
    DevBuf part(sizeof(double) * (size_t)pl.chunks * nn * pl.nj);
    DevBuf ones(sizeof(int) * nn);
    launch_fill<int>(ones.as<int>(), 0, nn, 1, 1, st);
    std::vector<double> unit((size_t)nn * Q);
    for (int q = 0; q < Q; ++q) {
      std::fill(unit.begin(), unit.end(), 0.0);
      for (int j = 0; j < nn; ++j) unit[(size_t)j * Q + q] = 1.0;
      RB_HIP(hipMemcpyAsync(th.p, unit.data(), sizeof(double) * unit.size(), hipMemcpyHostToDevice,
                            st));
      launch_coef_tables(g, nn, th.as<double>(), nullptr, coef.as<double>(), st);
      // V_j = A_q w_{j0+j}
      launch_apply(g, ld, nn, coef.as<double>(), bs->W64.as<double>() + (size_t)j0 * ld,
                   V.as<double>(), 0, nullptr, 0, nullptr, nullptr, nullptr, st);
      // t[j][i] = w_i^T V_j for i < n
      launch_projection(pl, RB_PREC_FP64, V.as<double>(), ld, bs->W64.p, ld, n, nn, ones.as<int>(),
                        part.p, st);
      launch_reduce_solve(true, part.p, pl.chunks, nn, pl.nj, n, nullptr, nullptr, nullptr,
                          t.as<double>(), nullptr, nullptr, 16, false, st);
      std::vector<double> th_((size_t)nn * n);
      RB_HIP(hipMemcpyAsync(th_.data(), t.p, sizeof(double) * th_.size(), hipMemcpyDeviceToHost,
                            st));
      RB_HIP(hipStreamSynchronize(st));
      for (int j = 0; j < nn; ++j)
        for (int i = 0; i < n; ++i) {
          const double v = th_[(size_t)j * n + i];
          AN[((size_t)q * n + i) * n + (j0 + j)] = v;
          AN[((size_t)q * n + (j0 + j)) * n + i] = v;
        }
    }
    // f_{N,r}: project the right-hand-side terms
    const ProjPlan pf = plan_projection(g.N, R, n, 2048);
    DevBuf partf(sizeof(double) * (size_t)pf.chunks * R * pf.nj);
    DevBuf tf(sizeof(double) * (size_t)R * n);
    DevBuf onesR(sizeof(int) * R);
    launch_fill<int>(onesR.as<int>(), 0, R, 1, 1, st);
    launch_projection(pf, RB_PREC_FP64, p->f.as<double>(), ld, bs->W64.p, ld, n, R,
                      onesR.as<int>(), partf.p, st);
    launch_reduce_solve(true, partf.p, pf.chunks, R, pf.nj, n, nullptr, nullptr, nullptr,
                        tf.as<double>(), nullptr, nullptr, 16, false, st);
    std::vector<double> fh((size_t)R * n);
    RB_HIP(hipMemcpyAsync(fh.data(), tf.p, sizeof(double) * fh.size(), hipMemcpyDeviceToHost, st));
    RB_HIP(hipStreamSynchronize(st));
    for (int r = 0; r < R; ++r)
      for (int j = j0; j < n; ++j) fN[(size_t)r * n + j] = fh[(size_t)r * n + j];
  }
  bs->AN_host = std::move(AN);
  bs->fN_host = std::move(fN);
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

static rb_basis* basis_upload(rb_ctx* ctx, const rb_problem* p, int n, const double* W) {
  auto bs = std::make_unique<rb_basis>();
  bs->ctx = ctx;
  bs->prob = p;
  bs->n = n;
  bs->ld = p->ld;
  bs->W64.alloc(sizeof(double) * ((size_t)basis_rows(n) * p->ld + kBasisTail));
  if (n > 0) {
    DevBuf nat(sizeof(double) * (size_t)n * p->N);
    RB_HIP(hipMemcpy(nat.p, W, sizeof(double) * (size_t)n * p->N, hipMemcpyHostToDevice));
    launch_to_storage(*p, n, nat.as<double>(), p->N, bs->W64.as<double>(), p->ld, ctx->stream);
    RB_HIP(hipStreamSynchronize(ctx->stream));
  }
  compute_reduced(bs.get(), 0);
  return bs.release();
}

}  // namespace rb

extern "C" {

rb_status rb_basis_from_host(rb_ctx* ctx, const rb_problem* p, int n, const double* W,
                             rb_basis** out) {
  return guarded([&] {
    RB_REQUIRE(ctx && p && out && n >= 0 && (n == 0 || W), RB_EINVAL, "bad basis arguments");
    RB_REQUIRE(n <= 80, RB_EUNSUPPORTED, "basis size above 80");
    check_finite(W, (size_t)n * p->N, "W");
    DeviceGuard dg(ctx->device);
    *out = basis_upload(ctx, p, n, W);
  });
}

rb_status rb_basis_info(const rb_basis* bs, int* n, double* W, double* AN, double* fN) {
  return guarded([&] {
    RB_REQUIRE(bs, RB_EINVAL, "null basis");
    const rb_problem* p = bs->prob;
    if (n) *n = bs->n;
    if (W && bs->n > 0) {
      DeviceGuard dg(bs->ctx->device);
      DevBuf nat(sizeof(double) * (size_t)bs->n * p->N);
      launch_from_storage(*p, bs->n, bs->W64.as<double>(), p->ld, nat.as<double>(), p->N,
                          bs->ctx->stream);
      RB_HIP(hipStreamSynchronize(bs->ctx->stream));
      RB_HIP(hipMemcpy(W, nat.p, sizeof(double) * (size_t)bs->n * p->N, hipMemcpyDeviceToHost));
    }
    if (AN) std::copy(bs->AN_host.begin(), bs->AN_host.end(), AN);
    if (fN) std::copy(bs->fN_host.begin(), bs->fN_host.end(), fN);
  });
}

static const uint64_t kMagic = 0x3142425242524231ull;  // "1BRBRBB1"

rb_status rb_basis_save(const rb_basis* bs, const char* path) {
  return guarded([&] {
    RB_REQUIRE(bs && path, RB_EINVAL, "null argument");
    const rb_problem* p = bs->prob;
    std::vector<double> W((size_t)bs->n * p->N);
    rb_status s = rb_basis_info(bs, nullptr, W.data(), nullptr, nullptr);
    RB_REQUIRE(s == RB_OK, s, rb_last_error());
    FILE* f = std::fopen(path, "wb");
    RB_REQUIRE(f, RB_EIO, std::string("cannot open ") + path);
    const int64_t hdr[6] = {(int64_t)kMagic, p->N, bs->n, p->g.Q, p->R, (int64_t)bs->picks.size()};
    bool ok = std::fwrite(hdr, sizeof(hdr), 1, f) == 1;
    ok = ok && std::fwrite(W.data(), sizeof(double), W.size(), f) == W.size();
    ok = ok && std::fwrite(bs->picks.data(), sizeof(int64_t), bs->picks.size(), f) ==
                   bs->picks.size();
    ok = ok && std::fwrite(bs->AN_host.data(), sizeof(double), bs->AN_host.size(), f) ==
                   bs->AN_host.size();
    ok = ok && std::fwrite(bs->fN_host.data(), sizeof(double), bs->fN_host.size(), f) ==
                   bs->fN_host.size();
    ok = (std::fclose(f) == 0) && ok;
    RB_REQUIRE(ok, RB_EIO, std::string("write failed: ") + path);
  });
}

rb_status rb_basis_load(rb_ctx* ctx, const rb_problem* p, const char* path, rb_basis** out) {
  return guarded([&] {
    RB_REQUIRE(ctx && p && path && out, RB_EINVAL, "null argument");
    FILE* f = std::fopen(path, "rb");
    RB_REQUIRE(f, RB_EIO, std::string("cannot open ") + path);
    int64_t hdr[6];
    bool ok = std::fread(hdr, sizeof(hdr), 1, f) == 1;
    if (!ok || (uint64_t)hdr[0] != kMagic) {
      std::fclose(f);
      throw Error{RB_EIO, "not a basis file"};
    }
    if (hdr[1] != p->N || hdr[3] != p->g.Q || hdr[4] != p->R || hdr[2] < 0 || hdr[2] > 80 ||
        hdr[5] < 0 || hdr[5] > hdr[2]) {
      std::fclose(f);
      throw Error{RB_EINVAL, "basis file does not match the problem"};
    }
    const int n = (int)hdr[2];
    std::vector<double> W((size_t)n * p->N);
    std::vector<int64_t> picks((size_t)hdr[5]);
    ok = std::fread(W.data(), sizeof(double), W.size(), f) == W.size();
    ok = ok && std::fread(picks.data(), sizeof(int64_t), picks.size(), f) == picks.size();
    std::fclose(f);
    RB_REQUIRE(ok, RB_EIO, "truncated basis file");
    DeviceGuard dg(ctx->device);
    rb_basis* bs = basis_upload(ctx, p, n, W.data());
    bs->picks = picks;
    *out = bs;
  });
}

rb_status rb_basis_destroy(rb_basis* bs) {
  return guarded([&] { delete bs; });
}

static void check_opts(const rb_solve_opts* o) {
  RB_REQUIRE(o && o->struct_size == sizeof(rb_solve_opts), RB_EINVAL,
             "rb_solve_opts.struct_size mismatch");
  RB_REQUIRE(o->rtol >= 0.0 && o->maxit >= 1 && o->fixed_iters >= 0, RB_EINVAL, "bad options");
  RB_REQUIRE(o->solver >= RB_SOLVER_RBCG && o->solver <= RB_SOLVER_CG, RB_EINVAL, "bad solver");
  RB_REQUIRE(o->precond_prec >= RB_PREC_FP64 && o->precond_prec <= RB_PREC_BF16, RB_EINVAL,
             "bad precision");
  RB_REQUIRE(o->smoother >= RB_SMOOTH_RBGS && o->smoother <= RB_SMOOTH_NONE, RB_EINVAL,
             "bad smoother");
  RB_REQUIRE(o->stencil_kind >= 0 && o->stencil_kind <= 4, RB_EINVAL, "bad stencil kind");
  RB_REQUIRE(std::isfinite(o->adapt_gamma) && o->adapt_gamma >= 0.0, RB_EINVAL,
             "bad adapt_gamma");
  RB_REQUIRE(o->adapt_gamma == 0.0 || o->solver == RB_SOLVER_RBCG, RB_EINVAL,
             "the adaptive basis size applies to RBCG only");
  RB_REQUIRE(o->smooth_sweeps >= 0 && o->smooth_sweeps <= 64, RB_EINVAL, "bad smooth_sweeps");
  RB_REQUIRE(o->residual_copy == 0 || o->residual_copy == 1, RB_EINVAL,
             "residual_copy must be 0 or 1");
  RB_REQUIRE(o->prolong_kind >= 0 && o->prolong_kind <= 2, RB_EINVAL,
             "prolong_kind must be 0, 1 or 2");
  RB_REQUIRE(o->paired_x_update == 0 || o->paired_x_update == 1, RB_EINVAL,
             "paired_x_update must be 0 or 1");
  RB_REQUIRE(std::isfinite(o->floor_factor) && o->floor_factor >= 0.0, RB_EINVAL,
             "bad floor_factor");
  RB_REQUIRE(o->smooth_sweeps <= 1 || o->smoother == RB_SMOOTH_RBGS ||
                 o->smoother == RB_SMOOTH_RBGS_SYM,
             RB_EUNSUPPORTED, "several sweeps need a Gauss-Seidel smoother");
}

rb_status rb_solve_batch(rb_ctx* ctx, const rb_problem* p, const rb_basis* bs,
                         const rb_solve_opts* o, int B, const double* theta, const double* phi,
                         const int* n_use, double* x, rb_query_stats* stats) {
  return guarded([&] {
    RB_REQUIRE(ctx && p && B >= 0 && B <= 65535, RB_EINVAL, "bad solve arguments");
    check_opts(o);
    RB_REQUIRE(bs || o->solver == RB_SOLVER_CG, RB_EINVAL, "basis required");
    RB_REQUIRE(!bs || bs->prob == p, RB_EINVAL, "basis belongs to another problem");
    if (B == 0) return;  // an empty batch: nothing to solve, nothing written
    RB_REQUIRE(theta && x && stats, RB_EINVAL, "bad solve arguments");
    check_finite(theta, (size_t)B * p->g.Q, "theta");
    if (phi) check_finite(phi, (size_t)B * p->R, "phi");
    DeviceGuard dg(ctx->device);
    BatchSolver s(ctx, p, bs, *o, B, theta, phi, n_use);
    s.run();
    std::vector<rb_query_stats> st;
    s.gather(x, p->N, st);
    std::copy(st.begin(), st.end(), stats);
  });
}

// Places a problem's queries in its batch so that those likely to need the most
// iterations (fewest basis vectors, then the largest spread of theta) fall into different
// groups of four consecutive queries: the batched passes work on such groups, and late in
// a solve, when few queries remain, they then keep many small blocks busy rather than a
// few full ones (1023^2, 242 queries of the uneven batch: 10.68 s against 11.02 s in the
// call's order and 13.79 s with the slow queries side by side).  Each query's result does
// not depend on its place.
static void spread_slow_queries(std::vector<int>& idx, const rb_query* qs, int Q, int nbasis) {
  const int B = (int)idx.size();
  if (B <= 4) return;
  std::vector<double> key_spread(B);
  std::vector<int> key_n(B);
  for (int k = 0; k < B; ++k) {
    const rb_query& q = qs[idx[k]];
    key_n[k] = q.n_use <= 0 ? nbasis : q.n_use;
    double lo = q.theta[0], hi = lo;
    for (int i = 1; i < Q; ++i) {
      lo = std::min(lo, q.theta[i]);
      hi = std::max(hi, q.theta[i]);
    }
    key_spread[k] = lo > 0.0 ? hi / lo : hi - lo;
  }
  std::vector<int> rank(B);
  for (int k = 0; k < B; ++k) rank[k] = k;
  std::stable_sort(rank.begin(), rank.end(), [&](int a, int b) {
    if (key_n[a] != key_n[b]) return key_n[a] < key_n[b];
    return key_spread[a] > key_spread[b];
  });
  // the r-th slowest goes to group r % G, slot r / G (G groups of four; the last group
  // may be short, so slots past B are skipped)
  const int G = (B + 3) / 4;
  std::vector<int> slot(4 * (size_t)G, -1);
  for (int r = 0; r < B; ++r) slot[(size_t)(r % G) * 4 + r / G] = idx[rank[r]];
  int k = 0;
  for (int v : slot)
    if (v >= 0) idx[k++] = v;
}

rb_status rb_solve_multi(rb_ctx* ctx, int nprob, const rb_problem* const* probs,
                         const rb_basis* const* bases, const rb_solve_opts* o, int B,
                         const rb_query* qs, rb_query_stats* stats) {
  return guarded([&] {
    RB_REQUIRE(ctx && probs && nprob >= 1 && B >= 0 && (B == 0 || (qs && stats)), RB_EINVAL,
               "bad multi-solve arguments");
    check_opts(o);
    // group the queries by problem; each group is one batched solver.  The groups run
    // concurrently, each on its own stream with its own workspace (the first group
    // uses the context's), and the host issues their iteration chunks round-robin.
    std::map<std::pair<int, double>, std::vector<int>> groups;
    for (int i = 0; i < B; ++i) {
      RB_REQUIRE(qs[i].problem >= 0 && qs[i].problem < nprob && qs[i].theta && qs[i].x,
                 RB_EINVAL, "bad query");
      RB_REQUIRE(std::isfinite(qs[i].rtol), RB_EINVAL, "bad query tolerance");
      RB_REQUIRE(probs[qs[i].problem], RB_EINVAL, "null problem");
      check_finite(qs[i].theta, (size_t)probs[qs[i].problem]->g.Q, "theta");
      const double tol = qs[i].rtol > 0.0 ? qs[i].rtol : o->rtol;
      groups[{qs[i].problem, tol}].push_back(i);
    }
    DeviceGuard dg(ctx->device);
    struct Group {
      const rb_problem* p;
      std::vector<int> idx;
      std::vector<double> th, ph;
      std::vector<int> nu;
      bool any_phi = false;
      hipStream_t st = nullptr;
      std::unique_ptr<BatchSolver> solver;
      bool running = false;
      rb_solve_opts opt;
    };
    std::vector<Group> gs;
    for (auto& kv : groups) {
      Group g;
      g.p = probs[kv.first.first];
      g.opt = *o;
      g.opt.rtol = kv.first.second;
      const rb_basis* bs = bases ? bases[kv.first.first] : nullptr;
      RB_REQUIRE(g.p, RB_EINVAL, "null problem");
      RB_REQUIRE(!bs || bs->prob == g.p, RB_EINVAL, "basis belongs to another problem");
      g.idx = kv.second;
      spread_slow_queries(g.idx, qs, g.p->g.Q, bs ? bs->n : 0);
      const int Bg = (int)g.idx.size();
      RB_REQUIRE(Bg <= 65535, RB_EINVAL, "more than 65535 queries on one problem and tolerance");
      const int Q = g.p->g.Q, R = g.p->R;
      g.th.resize((size_t)Bg * Q);
      g.ph.assign((size_t)Bg * R, 1.0);
      g.nu.resize(Bg);
      for (int k = 0; k < Bg; ++k) {
        const rb_query& q = qs[g.idx[k]];
        std::copy(q.theta, q.theta + Q, g.th.begin() + (size_t)k * Q);
        if (q.phi) {
          g.any_phi = true;
          std::copy(q.phi, q.phi + R, g.ph.begin() + (size_t)k * R);
        }
        g.nu[k] = (q.n_use <= 0 && bs) ? bs->n : q.n_use;
      }
      check_finite(g.th.data(), g.th.size(), "theta");
      gs.push_back(std::move(g));
    }
    // the first group runs on the context's stream and workspace, the others on the
    // context's group streams and workspaces (created on first use, kept for later calls)
    while (ctx->group_streams.size() + 1 < gs.size()) {
      hipStream_t st = nullptr;
      RB_HIP(hipStreamCreate(&st));  // blocking, default priority
      ctx->group_streams.push_back(st);
      ctx->group_ws.push_back(std::make_unique<Workspace>());
    }
    for (size_t i = 0; i < gs.size(); ++i)
      gs[i].st = i == 0 ? ctx->stream : ctx->group_streams[i - 1];
    for (size_t i = 0; i < gs.size(); ++i) {
      auto& g = gs[i];
      const rb_basis* bs = bases ? bases[g.idx.empty() ? 0 : qs[g.idx[0]].problem] : nullptr;
      Workspace* ws = i == 0 ? &ctx->ws : ctx->group_ws[i - 1].get();
      g.solver = std::make_unique<BatchSolver>(ctx, g.p, bs, g.opt, (int)g.idx.size(), g.th.data(),
                                               g.any_phi ? g.ph.data() : nullptr, g.nu.data(),
                                               g.st, ws);
      g.solver->start();
      g.running = true;
    }
    // each group issues its chunks (on large grids one more while the host reads the
    // flags of the chunk before it), then the host reads every running group's flags
    bool any = true;
    while (any) {
      for (auto& g : gs)
        if (g.running) g.solver->fill();
      any = false;
      for (auto& g : gs)
        if (g.running) {
          g.running = g.solver->poll();
          any |= g.running;
        }
    }
    for (size_t i = 0; i < gs.size(); ++i) {
      auto& g = gs[i];
      BatchSolver& sv = *g.solver;
      sv.finish();
      std::vector<rb_query_stats> st;
      Workspace* ws = i == 0 ? &ctx->ws : ctx->group_ws[i - 1].get();
      Buf xs = ws->get(WS_GATHER, sizeof(double) * g.idx.size() * g.p->N, sv.s());
      sv.gather(xs.as<double>(), g.p->N, st);
      for (size_t k = 0; k < g.idx.size(); ++k) {
        RB_HIP(hipMemcpyAsync(qs[g.idx[k]].x, xs.as<double>() + k * g.p->N,
                              sizeof(double) * g.p->N, hipMemcpyDeviceToDevice, sv.s()));
        stats[g.idx[k]] = st[k];
      }
      RB_HIP(hipStreamSynchronize(sv.s()));
    }
  });
}

rb_status rb_apply_batch(rb_ctx* ctx, const rb_problem* p, int B, const double* theta,
                         const double* u, double* y) {
  return guarded([&] {
    RB_REQUIRE(ctx && p && theta && u && y && B >= 1 && B <= 65535, RB_EINVAL, "bad arguments");
    check_finite(theta, (size_t)B * p->g.Q, "theta");
    DeviceGuard dg(ctx->device);
    hipStream_t st = ctx->stream;
    DevBuf th(sizeof(double) * (size_t)B * p->g.Q);
    RB_HIP(hipMemcpyAsync(th.p, theta, th.bytes, hipMemcpyHostToDevice, st));
    DevBuf coef(sizeof(double) * (size_t)B * p->g.ct_size);
    launch_coef_tables(p->g, B, th.as<double>(), nullptr, coef.as<double>(), st);
    DevBuf us(sizeof(double) * (size_t)B * p->ld), ys(sizeof(double) * (size_t)B * p->ld);
    launch_to_storage(*p, B, u, p->N, us.as<double>(), p->ld, st);
    launch_apply(p->g, p->ld, B, coef.as<double>(), us.as<double>(), ys.as<double>(), 0, nullptr,
                 0, nullptr, nullptr, nullptr, st);
    launch_from_storage(*p, B, ys.as<double>(), p->ld, y, p->N, st);
    RB_HIP(hipStreamSynchronize(st));
  });
}

rb_status rb_precond_batch(rb_ctx* ctx, const rb_problem* p, const rb_basis* bs,
                           const rb_solve_opts* o, int B, const double* theta, const int* n_use,
                           const double* r, double* y) {
  return guarded([&] {
    RB_REQUIRE(ctx && p && theta && r && y && B >= 1 && B <= 65535, RB_EINVAL, "bad arguments");
    check_opts(o);
    RB_REQUIRE(!bs || bs->prob == p, RB_EINVAL, "basis belongs to another problem");
    check_finite(theta, (size_t)B * p->g.Q, "theta");
    DeviceGuard dg(ctx->device);
    rb_solve_opts oo = *o;
    oo.solver = RB_SOLVER_RBCG;
    oo.beta_flexible = 0;
    BatchSolver s(ctx, p, bs, oo, B, theta, nullptr, n_use);
    s.prepare();
    set_stencil_tiles(s.tc);  // the requested stencil kinds (cached tiles, if any)
    hipStream_t st = ctx->stream;
    launch_to_storage(*p, B, r, p->N, s.r0.as<double>(), p->ld, st);
    s.factor();
    s.precondition(s.r0.as<double>(), nullptr);
    // y (FP64 or FP32) -> natural-order FP64
    DevBuf y64;
    const double* ysrc = s.y.as<double>();
    if (s.y32) {
      y64.alloc(sizeof(double) * (size_t)B * p->ld);
      launch_widen(s.y.as<float>(), y64.as<double>(), (int64_t)B * p->ld, st);
      ysrc = y64.as<double>();
    }
    launch_from_storage(*p, B, ysrc, p->ld, y, p->N, st);
    RB_HIP(hipStreamSynchronize(st));
    set_stencil_tiles(TuneConfig{});
  });
}

rb_status rb_project_batch(rb_ctx* ctx, const rb_problem* p, const rb_basis* bs, rb_prec prec,
                           int B, const double* r, double* t) {
  return guarded([&] {
    RB_REQUIRE(ctx && p && bs && r && t && B >= 1 && B <= 65535, RB_EINVAL, "bad arguments");
    RB_REQUIRE(bs->prob == p, RB_EINVAL, "basis belongs to another problem");
    RB_REQUIRE(prec >= RB_PREC_FP64 && prec <= RB_PREC_BF16, RB_EINVAL, "bad precision");
    DeviceGuard dg(ctx->device);
    hipStream_t st = ctx->stream;
    const int n = bs->n;
    if (n == 0) return;
    DevBuf rs(sizeof(double) * (size_t)B * p->ld);
    launch_to_storage(*p, B, r, p->N, rs.as<double>(), p->ld, st);
    const ProjPlan pl = plan_projection(p->g.N, B, n, 2048);
    const size_t acc = prec == RB_PREC_FP64 ? sizeof(double) : sizeof(float);
    DevBuf part(acc * (size_t)pl.chunks * B * pl.nj);
    DevBuf ones(sizeof(int) * B);
    launch_fill<int>(ones.as<int>(), 0, B, 1, 1, st);
    const void* W = const_cast<rb_basis*>(bs)->shadow(prec, st);
    launch_projection(pl, prec, rs.as<double>(), p->ld, W, p->ld, n, B, ones.as<int>(), part.p, st);
    DevBuf td(sizeof(double) * (size_t)B * n);
    launch_reduce_solve(prec == RB_PREC_FP64, part.p, pl.chunks, B, pl.nj, n, nullptr, nullptr,
                        nullptr, td.as<double>(), nullptr, nullptr, 16, false, st);
    RB_HIP(hipMemcpyAsync(t, td.p, sizeof(double) * (size_t)B * n, hipMemcpyDeviceToHost, st));
    RB_HIP(hipStreamSynchronize(st));
  });
}

rb_status rb_reduced_factor_batch(rb_ctx* ctx, const rb_basis* bs, int B, const double* theta,
                                  double* L, rb_status* status) {
  return guarded([&] {
    RB_REQUIRE(ctx && bs && theta && L && status && B >= 1 && B <= 65535, RB_EINVAL,
               "bad arguments");
    const int n = bs->n, Q = bs->prob->g.Q;
    RB_REQUIRE(n >= 1, RB_EINVAL, "empty basis");
    check_finite(theta, (size_t)B * Q, "theta");
    DeviceGuard dg(ctx->device);
    hipStream_t st = ctx->stream;
    DevBuf th(sizeof(double) * (size_t)B * Q), Ld(sizeof(double) * (size_t)B * n * n),
        sd(sizeof(int) * B);
    RB_HIP(hipMemcpyAsync(th.p, theta, th.bytes, hipMemcpyHostToDevice, st));
    launch_cholesky(bs->AN.as<double>(), n, Q, B, th.as<double>(), nullptr, Ld.as<double>(),
                    sd.as<int>(), st);
    std::vector<int> sh(B);
    RB_HIP(hipMemcpyAsync(L, Ld.p, Ld.bytes, hipMemcpyDeviceToHost, st));
    RB_HIP(hipMemcpyAsync(sh.data(), sd.p, sizeof(int) * B, hipMemcpyDeviceToHost, st));
    RB_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < B; ++i) status[i] = (rb_status)sh[i];
  });
}

}  // extern "C"
