// Launch declarations of the HIP kernels (stencil.hip, dense.hip, mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace rb {

// Per-query CG state on the device (each array has B entries).
struct QState {
  double* fnorm2;    // ||f_b||^2
  double* rho;       // y_k^T r_k
  double* alpha;
  double* beta;
  double* rel_rec;   // recursive relative residual
  double* rel_true;  // true relative residual (last check)
  double* scalar;    // scratch per query (e.g. ||r||^2 of RBI)
  int* active;
  int* status;
  int* iters;
  int* flag;     // true-residual check pending
  int* restart;  // next beta = 0 (p = y)
  // adaptive basis size (gamma2 > 0): nuse[b] grows by one, up to nmax, when
  // ||r_in||^2 < gamma2 ||r_new||^2, with rr_in the squared norm of the residual the
  // current direction was preconditioned from
  int* nuse = nullptr;
  double* rr_in = nullptr;
  double gamma2 = 0.0;
  int nmax = 0;
  int* at_floor = nullptr;  // accepted at the rounding level (floor test on)
  int* stalls = nullptr;    // true-residual checks in a row that gained less than half
  // paired x updates: alpha of an even iteration whose x update is still to be applied
  // (with that iteration's direction), 0 once applied; null when x is updated every
  // iteration
  double* apend = nullptr;
};

// Segments of a partial-sum buffer written by successive colour sweeps.
struct Segs {
  int n = 0;
  int cnt[kMaxColors];
  int64_t off[kMaxColors];
};

struct ProjPlan {
  bool wsplit = false;
  bool padded = false;  // R rows padded to a multiple of 64*qt (zero), W to round_up(n, 16)
  // wchunk: every wave covers all (at most 64) queries over a DOF range of its own, so
  // each basis row is read once per launch; chunks = 4 * blocks partial sums per query
  bool wchunk = false;
  int qt = 1, jt = 1, nj = 16;
  int qgroups = 1, chunks = 1, steps = 1;
  int blocks = 1;       // grid width (= chunks except in wchunk mode)
  int kend = 0;
};

// stencil.hip
// rows allocated for a basis of n vectors: padded so that the batched contraction
// kernels can read whole 16-row tiles plus one row of overrun without bounds checks;
// allocations add kBasisTail elements so a 256-node run may overrun the last row.
inline int basis_rows(int n) { return (n + 15) / 16 * 16 + 1; }
constexpr size_t kBasisTail = 1024;
// rows allocated for per-query vectors that the batched projection reads
inline int padded_queries(int B) { return (B + 255) / 256 * 256; }

// partial-sum chunks of a stencil pass over `count` storage positions
int stencil_chunks(int count);
// partial-sum chunks of an all-node stencil pass (apply, pass A/B, Jacobi)
int stencil_chunks_all(int N);
// partial-sum chunks of a one-colour sweep over storage positions [lo, hi) (its chunks
// start at lo rounded down to a 128-byte line; at most stencil_chunks(hi - lo) + 1)
int stencil_sweep_chunks(int lo, int hi);
// mode 1 with part2: partial sums of (|A| |u|)^2 as well (rounding level of the residual);
// y32 (mode 1, stencil grids): also an FP32 copy of y, rows of ld
void launch_apply(const StencilGeom& g, int64_t ld, int B, const double* coef, const double* u,
                  double* y, int mode, const double* rhs, int64_t rhs_ld, const double* rhs_scale,
                  const int* flag, double* part, hipStream_t s, double* part2 = nullptr,
                  float* y32 = nullptr);
// x_b += xc_b, xc_b = 0 for the queries with flag[b] != 0 (all of them if flag is null),
// over the ld entries of each row.  apend (nullable): an x update still to be applied,
// x_b += (xc_b + apend[b] p_b), for the queries with apend[b] != 0 (p rows of ld).
void launch_fold(const int* flag, int B, double* x, double* xc, int64_t ld, hipStream_t s,
                 const double* apend = nullptr, const double* p = nullptr);
// passes A and B return the number of partial sums per query they wrote (at most
// stencil_chunks_all(N); row stride stays stencil_chunks_all(N) in the solver's arrays)
template <typename TY>
int launch_pass_a(const StencilGeom& g, int64_t ld, int B, const double* coef, const TY* y,
                  int64_t y_ld, const double* p_old, double* p_new, const double* beta,
                  const int* active, double* part, hipStream_t s);
// whether the marching passes with qpb queries per block and zn nodes per thread can
// stage two plane buffers (within 64 KB of LDS)
bool zmarch_two_buffers(const StencilGeom& g, int B, int qpb, int zn);
// r32 (nullable, stencil grids): pass B also writes an FP32 copy of r_out (rows of ld).
// xd (stencil grids): the update of x, 0 x += alpha p, 1 none (deferred to the next
// iteration), 2 x = (x + a_prev p_prev) + alpha p (the deferred update first).
int launch_pass_b(const StencilGeom& g, int64_t ld, int B, const double* coef, const double* p,
                  double* x, const double* r_in, double* r_out, const double* alpha,
                  const int* active, double* part, hipStream_t s, float* r32 = nullptr,
                  int xd = 0, const double* p_prev = nullptr, const double* a_prev = nullptr);
// returns the number of partial sums per query it wrote (row stride of part0 / part1;
// at most stencil_chunks of the colour's node count).  RT = float (TY = float, stencil
// grids): rhs is an FP32 copy of the right-hand side; the same y, since the update rounds
// rhs to FP32 first.
template <typename TY, typename RT = double>
int launch_gs_color(const StencilGeom& g, int color, int B, const double* coef, TY* y,
                    int64_t y_ld, const RT* rhs, int64_t rhs_ld, const double* rhs_scale,
                    const double* rhs2, int64_t rhs2_ld, const int* active, double* part0,
                    double* part1, hipStream_t s);
// One forward red-black sweep y = S(A, rhs, z) in one launch marching along z, for a start
// z that is zero on the red nodes, read from the black half of zs (not written; y is
// written on both colours).  Same y as the two launch_gs_color sweeps.  3D stencil grids
// with nx <= 255 only (gs_fused_supported); returns the number of partial sums per query
// (<= cap), 0 if not run.
bool gs_fused_supported(const StencilGeom& g);
template <typename TY>
int launch_gs_fused(const StencilGeom& g, int B, const double* coef, const TY* zs, TY* y,
                    int64_t y_ld, const double* rhs, int64_t rhs_ld, const double* rhs2,
                    int64_t rhs2_ld, const int* active, double* part0, double* part1, int cap,
                    hipStream_t s);
template <typename TY>
void launch_jacobi(const StencilGeom& g, int B, const double* coef, const TY* z, TY* y,
                   int64_t y_ld, double omega, const double* rhs, int64_t rhs_ld,
                   const double* rhs2, int64_t rhs2_ld, const int* active, double* part0,
                   double* part1, hipStream_t s);

// csr.hip: the same passes for general sparse problems (the stencil launchers above
// forward to these when g.csr is set)
int csr_chunks(int rows);
void csr_coef_tables(const StencilGeom& g, int B, const double* theta, const int* qidx,
                     double* coef, hipStream_t s);
void csr_apply(const StencilGeom& g, int64_t ld, int B, const double* coef, const double* u,
               double* y, int mode, const double* rhs, int64_t rhs_ld, const double* rhs_scale,
               const int* flag, double* part, hipStream_t s, double* part2 = nullptr);
template <typename TY>
int csr_pass_a(const StencilGeom& g, int64_t ld, int B, const double* coef, const TY* y,
               int64_t y_ld, const double* p_old, double* p_new, const double* beta,
               const int* active, double* part, hipStream_t s);
int csr_pass_b(const StencilGeom& g, int64_t ld, int B, const double* coef, const double* p,
               double* x, const double* r_in, double* r_out, const double* alpha,
               const int* active, double* part, hipStream_t s);
template <typename TY>
void csr_gs_color(const StencilGeom& g, int color, int B, const double* coef, TY* y,
                  int64_t y_ld, const double* rhs, int64_t rhs_ld, const double* rhs_scale,
                  const double* rhs2, int64_t rhs2_ld, const int* active, double* part0,
                  double* part1, hipStream_t s);
template <typename TY>
void csr_jacobi(const StencilGeom& g, int B, const double* coef, const TY* z, TY* y,
                int64_t y_ld, double omega, const double* rhs, int64_t rhs_ld,
                const double* rhs2, int64_t rhs2_ld, const int* active, double* part0,
                double* part1, hipStream_t s);
void csr_to_storage(int N, const int* perm, int B, const double* nat, int64_t nat_ld,
                    double* sto, int64_t sto_ld, hipStream_t s);
void csr_from_storage(int N, const int* perm, int B, const double* sto, int64_t sto_ld,
                      double* nat, int64_t nat_ld, hipStream_t s);

// dense.hip
ProjPlan plan_projection(int N, int B, int n, int target_blocks);
// Turns a padded batched plan for 16 < B <= 64 queries and n > 48 basis vectors (FP32 or
// BF16 basis) into wchunk mode with about 2 * target_blocks waves; other plans are
// unchanged.
void plan_wave_chunks(ProjPlan& p, int B, int target_blocks, rb_prec prec);
// qlist (nullable; the batched path only): active queries in increasing order with their
// count in qlist[B] (launch_compact_active); rows of other queries are then not read.
// R32 (nullable; FP32 / BF16 basis): an FP32 copy of R with the same layout, read instead
// of R (the same partial sums: the products round R to FP32 first).
void launch_projection(const ProjPlan& pl, rb_prec prec, const double* R, int64_t r_ld,
                       const void* W, int64_t w_ld, int n, int B, const int* active, void* part,
                       hipStream_t s, const int* qlist = nullptr, const float* R32 = nullptr);
// MFMA path (FP32/BF16, B >= 16): e must have round_up(B, 64) rows, zero beyond B, and
// W basis_rows(n) rows plus kBasisTail elements, zero beyond n.
// qlist as for launch_projection (MFMA path only)
void launch_prolong(rb_prec prec, const void* W, int64_t w_ld, int n, const double* e64,
                    const float* e32, int e_ld, int B, const int* active, void* out,
                    bool out_is_double, int64_t o_ld, int lo, int hi, bool add, hipStream_t s,
                    const int* qlist = nullptr);
// qlist[B + 1]: the indices of the active queries in increasing order, then their count
void launch_compact_active(const int* active, int B, int* qlist, hipStream_t s);
// out[b] = sum_r phi[b][r] f_r over the R right-hand-side terms f (rows of ld, storage
// order); B rows of ld, zero beyond N
void launch_combine_rhs(const double* f, int64_t ld, int R, const double* phi, int B, int N,
                        double* out, hipStream_t s);
void launch_cholesky(const double* AN, int n, int Q, int B, const double* theta, const int* n_use,
                     double* L, int* status, hipStream_t s);
void launch_reduce_solve(bool fp64_part, const void* part, int chunks, int B, int nj, int n,
                         const int* n_use, const double* L, const int* active, double* t_out,
                         double* e64, float* e32, int e_ld, bool solve, hipStream_t s);
void launch_fin_alpha(const double* part, int stride, int cnt, const QState& q, int B,
                      hipStream_t s);
// defer: pass B left this iteration's x update to the next one; q.apend (if set) then
// takes alpha of the queries active in it, else 0
void launch_fin_rr(const double* part, int stride, int cnt, const QState& q, int B, double rtol,
                   int maxit, bool fixed, hipStream_t s, bool defer = false);
// part2 (nullable): partial sums of (|A||x|)^2; floor_factor > 0 also accepts residuals
// within floor_factor * eps * || |A||x| || (at_floor)
void launch_fin_true(const double* part, int stride, int cnt, const QState& q, int B, double rtol,
                     int maxit, hipStream_t s, const double* part2 = nullptr,
                     double floor_factor = 0.0);
// Partial sums of y^T r (pr) and y^T r_old (fr): segment c is [B][cnt[c]] starting at
// element off[c]; the segments are summed in order.
void launch_fin_beta(const double* pr, const double* fr, const Segs& sg, const QState& q, int B,
                     bool flexible, hipStream_t s);
void launch_fin_sum(const double* part, int stride, int cnt, double* out, const int* active,
                    int B, hipStream_t s);
template <typename T>
void launch_fill(T* dst, int64_t ld, int64_t n, int B, T value, hipStream_t s);
// returns the number of partial sums per query; r32 (nullable): also an FP32 copy of r
int launch_init_rhs(const double* f, int64_t f_ld, const double* scale, int N, double* r,
                    int64_t ld, int B, double* part, int per_thread, hipStream_t s,
                    float* r32 = nullptr);
void launch_cast(const double* src, void* dst, int64_t n, rb_prec prec, hipStream_t s);
void launch_widen(const float* src, double* dst, int64_t n, hipStream_t s);
void compute_reduced(rb_basis* bs, int j0);
void launch_sweep_coeffs(const double* AN, const double* fN, int n, int Q, int R, int M,
                         const double* theta, const double* phi, double* a, int a_ld, double* l1,
                         int* status, hipStream_t s);
void launch_argmax(const double* v, const int* excluded, int M, double* out_val, int* out_idx,
                   int* nan_flag, hipStream_t s);
// returns the number of chunks (partials per row)
int launch_dot(const double* a, const double* c, int64_t ld, int N, int B, double* part,
               int per_thread, hipStream_t s);
void launch_scale(double* dst, const double* src, int64_t n, double alpha, hipStream_t s);

}  // namespace rb
