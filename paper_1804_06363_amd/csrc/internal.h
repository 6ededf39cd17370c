// Internal types of librb: context, problem, basis, launch declarations.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <exception>
#include <new>
#include <string>
#include <memory>
#include <vector>

#include "../../include/rb.h"
#include "common.h"

namespace rb {

// ---- error handling --------------------------------------------------------
void set_error(const std::string& msg);
struct Error {
  rb_status code;
  std::string msg;
};
#define RB_HIP(call)                                                                \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess)                                                           \
      throw ::rb::Error{RB_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)
#define RB_REQUIRE(cond, code, msg)                      \
  do {                                                   \
    if (!(cond)) throw ::rb::Error{(code), (msg)};       \
  } while (0)

// Device allocation owned by a C++ object; throws RB_ENOMEM on failure.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t n) { alloc(n); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t n);
  void release();
  template <typename T> T* as() const { return reinterpret_cast<T*>(p); }
};

// Makes `dev` the calling thread's current device for the guard's lifetime and restores
// the previous one on every exit path (including exceptions).
struct DeviceGuard {
  int old = 0;
  explicit DeviceGuard(int dev) {
    (void)hipGetDevice(&old);
    if (old != dev) RB_HIP(hipSetDevice(dev));
  }
  ~DeviceGuard() { (void)hipSetDevice(old); }
};

// Runs an entry point's body: RB_OK, or the status and message of whatever it threw.
template <typename F>
inline rb_status guarded(F&& f) {
  try {
    f();
    return RB_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return RB_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return RB_EINVAL;
  } catch (...) {
    set_error("unknown error");
    return RB_EINVAL;
  }
}

inline void check_finite(const double* v, size_t n, const char* what) {
  for (size_t i = 0; i < n; ++i)
    RB_REQUIRE(std::isfinite(v[i]), RB_EINVAL, std::string(what) + " contains NaN or Inf");
}

// The fixed device buffer of the entry points that allocate nothing: resolves its
// address on `device` (the current device) once; called when a context is created.
void noalloc_attach(int device);

}  // namespace rb

// ---- stencil geometry (device-side view) --------------------------------------
// Vectors of a stencil problem are stored in red-black order: position g < NR holds
// the red node with lexicographic index L = 2g, position g >= NR the black node
// L = 2(g - NR) + 1.  With n_x (and n_y in 3D) odd, the parity of L equals the
// colour (i + j + k) mod 2.
constexpr int kMaxColors = 32;  // colour classes of the Gauss-Seidel smoother

struct StencilGeom {
  int dim;
  int nx, ny, nz;
  int bx, by, bz;
  int Q;
  int N;      // nodes
  int NR;     // red nodes = (N + 1) / 2
  int nxy;    // nx * ny
  rbk::FastDiv div_nx, div_nxy;
  // per-axis node tables (device): packed state | lo-face block << 8 | hi-face block << 16
  const uint32_t* tab[3];
  // coefficient-table layout per query (doubles)
  int ct_off[3];  // offset of the table of axis a
  int ct_s1[3];   // size of the first tangential state dimension (or 1)
  int ct_s2[3];   // size of the second tangential state dimension (or 1)
  int ct_size;    // doubles per query (padded)
  // colour classes of the Gauss-Seidel smoother in storage order: class c holds the
  // positions [coff[c], coff[c+1]); the grids use red-black (C = 2, coff[1] = NR)
  int C;
  int coff[kMaxColors + 1];
  // general sparse problems (csr != 0): terms on a shared pattern in sliced ELL form,
  // rows in storage (colour-major) order.  Slice s holds rows [64 s, 64 s + 64);
  // entry k of its lane l is at sptr[s] + 64 k + l (column in scol, storage index; the
  // value of term q in sval[q * sval_ld + ...]); the diagonal is kept apart in diag[q * N
  // + row] and padding entries point at their own row with value 0.
  int csr;
  const int64_t* sptr;
  const int* scol;
  const double* sval;
  int64_t sval_ld;
  const double* diag;
};

namespace rb {
// Per-kernel timing with HIP events on the context's stream (off by default).
struct Profiler {
  bool on = false;
  struct Pending {
    const char* name;
    hipEvent_t a, b;
  };
  struct Total {
    double ms = 0.0;
    int64_t launches = 0;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<std::string, Total>> totals;
  hipEvent_t get();
  void record(const char* name, hipEvent_t a, hipEvent_t b) { pending.push_back({name, a, b}); }
  void resolve();  // completed pairs (the others stay pending)
  ~Profiler();
};
}  // namespace rb

namespace rb {
// Non-owning view of a device buffer.
struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
  template <typename T> T* as() const { return reinterpret_cast<T*>(p); }
};
// Tile choices of the batched kernels (0 = built-in heuristic), per solve.
struct TuneConfig {
  int qpb_a = 0, qpb_b = 0, qpb_gs = 0;  // queries per block of pass A / pass B / sweeps
  int proj_target = 0;                   // projection: target number of blocks
  int kind_a = 0, kind_b = 0;            // pass A / B: 0 default, 1 chunked, 2 z-marching
  int kind_gs = 0;                       // colour sweeps: the same kinds
  int kind_pro = 0;                      // batched prolongation: 0 default (MFMA), 1 MFMA,
                                         // 2 vector units
  int zn_a = 0, zn_b = 0;                // marching passes A / B: nodes per thread (0 = 2)
  int np_gs = 0;                         // marching sweeps: column pairs per thread (0 = 2)
  int nb_b = 0;                          // marching pass B: LDS plane buffers, 1 or 2 (0 =
                                         // 2 where they fit in 64 KB)
  int nb_a = 0;                          // marching pass A: the same (0 = 1)
};
// Autotuner cache: key -> choice; persisted as JSON when RB_AUTOTUNE_CACHE names a file.
struct Tuner {
  bool loaded = false;
  std::string path;
  std::vector<std::pair<std::string, TuneConfig>> table;
  const TuneConfig* find(const std::string& key) const;
  void put(const std::string& key, const TuneConfig& c);
  void load();
  void save() const;
};
// Tiles the stencil launchers use on the calling thread (set by the solver).
void set_stencil_tiles(const TuneConfig& c);
TuneConfig stencil_tiles();

enum WsSlot {
  WS_THETA, WS_SCALE, WS_NUSE, WS_COEF, WS_L, WS_E64, WS_E32, WS_PROJ, WS_X, WS_R0, WS_R1,
  WS_P0, WS_P1, WS_Y, WS_Z, WS_PM, WS_PM2, WS_PR0, WS_PR1, WS_Q, WS_QLIST, WS_FB, WS_PHI,
  WS_GATHER, WS_ONES, WS_XC, WS_R32, WS_COUNT
};
}  // namespace rb

namespace rb {
// Solver workspace, grown on demand.  Contents are not preserved between solves.
struct Workspace {
  DevBuf slot[WS_COUNT];
  Buf get(int i, size_t bytes, hipStream_t s) {
    if (slot[i].bytes < bytes) {
      (void)hipStreamSynchronize(s);
      slot[i].alloc(bytes);
    }
    return Buf{slot[i].p, slot[i].bytes};
  }
};
}  // namespace rb

struct rb_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipDeviceProp_t prop{};
  rb::Profiler prof;
  rb::Tuner tuner;
  // the context's workspace, kept until the context is destroyed (one solver at a time
  // uses it; concurrent groups of rb_solve_multi get their own)
  rb::Workspace ws;
  rb::Buf get_ws(int slot, size_t bytes) { return ws.get(slot, bytes, stream); }
  // streams and workspaces of the further groups of rb_solve_multi, grown on demand and
  // kept for later calls until the context is destroyed
  std::vector<hipStream_t> group_streams;
  std::vector<std::unique_ptr<rb::Workspace>> group_ws;
};

namespace rb {
// Times the launches issued while it is alive (when profiling is on and the stream is
// not being captured into a graph).
struct ProfScope {
  rb_ctx* ctx;
  const char* name;
  hipEvent_t a = nullptr;
  // timing only on the context's own stream
  ProfScope(rb_ctx* c, const char* n, hipStream_t on = nullptr) : ctx(c), name(n) {
    if (!ctx->prof.on || (on && on != ctx->stream)) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(ctx->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
      return;
    a = ctx->prof.get();
    (void)hipEventRecord(a, ctx->stream);
  }
  ~ProfScope() {
    if (!a) return;
    hipEvent_t b = ctx->prof.get();
    (void)hipEventRecord(b, ctx->stream);
    ctx->prof.record(name, a, b);
  }
};
}  // namespace rb

struct rb_problem {
  rb_ctx* ctx = nullptr;
  rb_stencil_desc desc{};
  StencilGeom g{};
  int64_t N = 0;
  int64_t ld = 0;  // padded per-vector stride (elements)
  int R = 1;
  rb::DevBuf tabs;       // per-axis node tables
  rb::DevBuf perm;       // int32 [N]: storage position -> natural index (sparse problems)
  std::vector<int> perm_h;  // the same on the host (sparse problems)
  std::vector<int> color_h; // colour class of every unknown, natural order (sparse problems)
  rb::DevBuf sptr, scol, sval, diag;  // sliced ELL terms (sparse problems)
  // natural index of storage position pos
  int nat_index(int pos) const {
    if (g.csr) return perm_h[pos];
    return pos < g.NR ? 2 * pos : 2 * (pos - g.NR) + 1;
  }
  rb::DevBuf f;          // double [R][ld], storage (red-black) order
};

struct rb_basis {
  rb_ctx* ctx = nullptr;
  const rb_problem* prob = nullptr;
  int n = 0;
  int cap = 0;      // columns W64 has room for (n_max while the greedy grows it)
  int64_t ld = 0;
  rb::DevBuf W64;   // double [n][ld] storage order
  rb::DevBuf W32;   // float  [n][ld] shadow (built on first use, extended as n grows)
  rb::DevBuf W16;   // bf16   [n][ld] shadow (likewise)
  int n32 = 0, n16 = 0;  // columns converted into W32 / W16
  rb::DevBuf AN;    // double [Q][n][n]
  rb::DevBuf fN;    // double [R][n]
  std::vector<double> AN_host, fN_host;
  std::vector<int64_t> picks;
  // the latest cast into a shadow and the stream it ran on: a consumer on another
  // stream waits for it
  hipEvent_t cast_done = nullptr;
  hipStream_t cast_stream = nullptr;
  // the basis in precision `prec` for kernels issued on `consumer` (converting the
  // columns not converted yet, stream-ordered before the consumer's later work)
  const void* shadow(rb_prec prec, hipStream_t consumer);
  rb_basis() = default;
  rb_basis(const rb_basis&) = delete;
  rb_basis& operator=(const rb_basis&) = delete;
  ~rb_basis() {
    if (cast_done) (void)hipEventDestroy(cast_done);
  }
};

namespace rb {

// ---- launchers (kernels in *.hip) ---------------------------------------------
// problem setup
void launch_coef_tables(const StencilGeom& g, int B, const double* theta, const int* qidx,
                        double* coef, hipStream_t s);
void launch_to_storage(const rb_problem& p, int B, const double* nat, int64_t nat_ld,
                       double* sto, int64_t sto_ld, hipStream_t s);
void launch_from_storage(const rb_problem& p, int B, const double* sto, int64_t sto_ld,
                         double* nat, int64_t nat_ld, hipStream_t s);

}  // namespace rb
