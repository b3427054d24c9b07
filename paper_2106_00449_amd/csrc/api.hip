// C ABI of libgdc: handle set-up, the mobility operators, the device GMRES
// driver and the gDC / Euler-Maruyama step orchestration.
//
// Everything per step runs on the handle's stream; the host reads back only
// the GMRES Hessenberg column of each iteration (to decide convergence) and
// the step's drift factor nu for the statistics.

#include "gdc_internal.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>

namespace gdc {

namespace {
thread_local std::string g_last_error;
}

// Staging memory of gdc_philox_normals_noalloc: a file-scope device array,
// one copy per GPU, held until the process ends.  Host code never uses the
// array's name as an address (on the host it is only a stand-in for the
// symbol); it uses the device address looked up per device below.
constexpr int NOALLOC_MAX_NORMAL_GROUPS = 65536;   // 4 normals each: 2 MiB
static __device__ __align__(256) double scratch[4 * NOALLOC_MAX_NORMAL_GROUPS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

// Device address of `scratch` on `device`, looked up once per device with
// that device current (every GPU holds its own copy at its own address).
int scratch_address(int device, void** out) {
  if (device < 0 || device >= MAX_DEVICES) {
    set_error("device ordinal out of range for the staging array");
    return GDC_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    hipError_t e = hipSetDevice(device);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev >= 0) (void)hipSetDevice(prev);
    if (e != hipSuccess || !p) {
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return GDC_EDEVICE;
    }
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return GDC_OK;
}

void set_error(const std::string& msg) { g_last_error = msg; }

namespace {
struct Probe {
  std::string family;
  std::vector<hipEvent_t> ev;   // pairs: start, stop
  size_t used = 0;
  long long dropped = 0;
};
Probe g_probe;
constexpr size_t PROBE_PAIRS = 8192;
}  // namespace

ProbeEvents probe_claim(const char* family) {
  ProbeEvents pe;
  if (g_probe.family.empty() || g_probe.family != family) return pe;
  if (g_probe.used + 2 > g_probe.ev.size()) {
    ++g_probe.dropped;
    return pe;
  }
  pe.start = g_probe.ev[g_probe.used];
  pe.stop = g_probe.ev[g_probe.used + 1];
  g_probe.used += 2;
  return pe;
}

bool probe_active() { return !g_probe.family.empty(); }

int check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("launch of ") + what + ": " + hipGetErrorString(e));
    return GDC_EDEVICE;
  }
  return GDC_OK;
}

namespace {

constexpr int HCOLS = 64;       // device scratch per Hessenberg column section
constexpr double PINV_RCOND = 1e-10;

// ------------------------------------------------------------ host linear algebra

// Symmetric eigen-decomposition by cyclic Jacobi rotations (n small).
void jacobi_eigen(int n, std::vector<double> A, std::vector<double>& evals, std::vector<double>& evecs) {
  evecs.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) evecs[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += A[i * n + j] * A[i * n + j];
        if (i != j) off += A[i * n + j] * A[i * n + j];
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // A <- J^T A J
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = evecs[k * n + p], vkq = evecs[k * n + q];
          evecs[k * n + p] = c * vkp - s * vkq;
          evecs[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  evals.resize(n);
  for (int i = 0; i < n; ++i) evals[i] = A[i * n + i];
}

// Inverse by Gauss-Jordan elimination with partial pivoting; false if singular.
bool invert(int n, std::vector<double> A, std::vector<double>& inv) {
  inv.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (std::fabs(A[piv * n + c]) < 1e-300) return false;
    if (piv != c)
      for (int k = 0; k < n; ++k) {
        std::swap(A[c * n + k], A[piv * n + k]);
        std::swap(inv[c * n + k], inv[piv * n + k]);
      }
    const double d = 1.0 / A[c * n + c];
    for (int k = 0; k < n; ++k) {
      A[c * n + k] *= d;
      inv[c * n + k] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        A[r * n + k] -= f * A[c * n + k];
        inv[r * n + k] -= f * inv[c * n + k];
      }
    }
  }
  return true;
}

// Unbounded RPY tensor for equal radii a at separation d (3x3 row-major).
void rpy(const double* d, double a, double eta, double* T) {
  const double r = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const double pi = 3.14159265358979323846;
  if (r == 0.0) {
    for (int k = 0; k < 9; ++k) T[k] = (k % 4 == 0) ? 1.0 / (6.0 * pi * eta * a) : 0.0;
    return;
  }
  double ci, cr;
  if (r >= 2.0 * a) {
    ci = (1.0 + 2.0 * a * a / (3.0 * r * r)) / (8.0 * pi * eta * r);
    cr = (1.0 - 2.0 * a * a / (r * r)) / (8.0 * pi * eta * r);
  } else {
    ci = (1.0 - 9.0 * r / (32.0 * a)) / (6.0 * pi * eta * a);
    cr = (3.0 * r / (32.0 * a)) / (6.0 * pi * eta * a);
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) T[3 * i + j] = (i == j ? ci : 0.0) + cr * d[i] * d[j] / (r * r);
}

struct ShapeHost {
  int nb = 0;
  std::vector<double> b;       // nb x 3
  double Lp = 0.0;
  double pinv[36];
  double null[36];
  bool has_null = false;
  std::vector<double> precT;   // D x D transposed inverse, D = 3 nb + 6
};

// Builds K^T K (body frame), its pseudo-inverse, the null-space projector and
// the inverse of the preconditioner block [[M_RPY, -K], [-K^T, -Pi]].
bool build_shape(ShapeHost& S, double a, double eta, std::string& err) {
  const int nb = S.nb;
  std::vector<double> A(36, 0.0);
  for (int i = 0; i < nb; ++i) {
    const double* r = &S.b[3 * i];
    // K_i = [I, [x r]]  with [x r] = -[r x]
    double Ki[18];
    for (int k = 0; k < 18; ++k) Ki[k] = 0.0;
    for (int k = 0; k < 3; ++k) Ki[6 * k + k] = 1.0;
    const double cx[9] = {0, -r[2], r[1], r[2], 0, -r[0], -r[1], r[0], 0};  // [r x]
    for (int row = 0; row < 3; ++row)
      for (int col = 0; col < 3; ++col) Ki[6 * row + 3 + col] = -cx[3 * row + col];
    for (int p = 0; p < 6; ++p)
      for (int q = 0; q < 6; ++q)
        for (int k = 0; k < 3; ++k) A[6 * p + q] += Ki[6 * k + p] * Ki[6 * k + q];
  }
  std::vector<double> ev, V;
  jacobi_eigen(6, A, ev, V);
  double emax = 0.0;
  for (double e : ev) emax = std::max(emax, std::fabs(e));
  for (int k = 0; k < 36; ++k) S.pinv[k] = S.null[k] = 0.0;
  for (int m = 0; m < 6; ++m) {
    const bool keep = ev[m] > PINV_RCOND * emax;
    if (!keep) S.has_null = true;
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) {
        const double vv = V[i * 6 + m] * V[j * 6 + m];
        if (keep)
          S.pinv[6 * i + j] += vv / ev[m];
        else
          S.null[6 * i + j] += vv;
      }
  }
  double Lp = 0.0;
  for (int i = 0; i < nb; ++i)
    for (int j = i + 1; j < nb; ++j) {
      double d2 = 0.0;
      for (int k = 0; k < 3; ++k) d2 += (S.b[3 * i + k] - S.b[3 * j + k]) * (S.b[3 * i + k] - S.b[3 * j + k]);
      Lp = std::max(Lp, std::sqrt(d2));
    }
  S.Lp = nb < 2 ? a : Lp;
  const int D = 3 * nb + 6;
  std::vector<double> P(D * D, 0.0);
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < nb; ++j) {
      double d[3] = {S.b[3 * i] - S.b[3 * j], S.b[3 * i + 1] - S.b[3 * j + 1], S.b[3 * i + 2] - S.b[3 * j + 2]};
      double T[9];
      rpy(d, a, eta, T);
      for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) P[(3 * i + p) * D + 3 * j + q] = T[3 * p + q];
    }
  for (int i = 0; i < nb; ++i) {
    const double* r = &S.b[3 * i];
    const double cx[9] = {0, -r[2], r[1], r[2], 0, -r[0], -r[1], r[0], 0};
    for (int k = 0; k < 3; ++k) {
      P[(3 * i + k) * D + 3 * nb + k] = -1.0;
      P[(3 * nb + k) * D + 3 * i + k] = -1.0;
      for (int c = 0; c < 3; ++c) {
        // -K: -[x r] = [r x];  -K^T: ([r x])^T
        P[(3 * i + k) * D + 3 * nb + 3 + c] = cx[3 * k + c];
        P[(3 * nb + 3 + c) * D + 3 * i + k] = cx[3 * k + c];
      }
    }
  }
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) P[(3 * nb + i) * D + 3 * nb + j] = -S.null[6 * i + j];
  std::vector<double> inv;
  if (!invert(D, P, inv)) {
    err = "singular preconditioner block";
    return false;
  }
  S.precT.assign(D * D, 0.0);
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) S.precT[j * D + i] = inv[i * D + j];
  return true;
}

template <typename T>
int dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  const hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
    return GDC_ENOMEM;
  }
  return GDC_OK;
}

struct GmresResult {
  int its = 0;
  double relres = 0.0;
  bool converged = false;
};

// Status of the device GMRES as the host reads it.
struct GmStatus {
  double est;
  int its, kdone, done, converged;
};

// Host side of a GMRES solve in progress (the device side is GmresState).
// A solve advances by one enqueue or one status read at a time, so that one
// host thread can keep the solves of many handles in flight at once.
struct SolveRun {
  enum Phase { IDLE, CYCLE, ITER, FINISH, FINISH_WAIT, DONE };
  Phase phase = IDLE;
  const double *Y = nullptr, *q = nullptr, *r = nullptr;
  bool first = true;    // first cycle: the residual is the right-hand side
  int k = 0;            // Arnoldi column of the current cycle
  bool queued = false;  // iteration k is on the stream
  bool deferred = false;  // iteration k waits for a launch fused with other suspensions
  GmStatus st{};
  GmresResult res{};
};

// Host side of the time steps in progress: the pre-solve kernels are queued
// on entry to SOLVE, the update and the readback when the solve is done.
// Steps are pipelined: once a step's update is queued, the next step's
// work is queued at once, and the step's readback (nu, error flags, sine
// amplitude) is read from one of two pinned slots when it has landed, so the
// GPU does not idle between steps while the host reads and enqueues.
struct StepRun {
  enum Phase { IDLE, SOLVE };
  Phase phase = IDLE;
  int to_start = 0;          // steps the driver still wants started
  int pend = 0;              // queued steps whose readback is outstanding (<= 2)
  int head = 0;              // slot of the oldest outstanding readback
  GmresResult slot_gr[2]{};  // solve statistics of the step in each slot
  GmresResult gr{};          // of the last completed step
  double nu = 1.0;           // of the last completed step
};

// Outcome of one advance of a solve or a step.
enum Advance { ADV_BLOCKED = 0, ADV_PROGRESS = 1, ADV_DONE = 2 };

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace
}  // namespace gdc

using namespace gdc;

struct gdc_handle {
  gdc_config cfg{};
  int N = 0, M = 0;
  int Ms = 0;           // spreading blobs: M, or 2M in the slip channel (the images M .. 2M - 1)
  long long nx = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int precision = GDC_FP32;
  size_t rsize = 4;
  uint64_t step = 0;
  GridGeom geom{};
  int maxdim = 0;
  int restart = 50, maxit = 200;
  double tol = 1e-6;
  int nc[3] = {0, 0, 0};
  int cell_cap = 0;
  std::vector<ShapeHost> shapes;
  std::vector<int> body_shape;

  std::vector<void*> allocs;
  void* grid[3] = {nullptr, nullptr, nullptr};
  void* grid_fl = nullptr;
  void* tw[3] = {nullptr, nullptr, nullptr};
  BodyTables bt{};
  double *Y = nullptr, *q = nullptr, *Ym = nullptr, *qm = nullptr, *r = nullptr, *rm = nullptr;
  double *v = nullptr, *vd = nullptr, *dr = nullptr, *wrfd = nullptr, *calV = nullptr, *dp = nullptr, *nu = nullptr;
  double *F = nullptr, *fblob = nullptr, *cforce = nullptr, *io = nullptr;
  int *cell_count = nullptr, *cell_list = nullptr, *flags = nullptr;
  double *Vb = nullptr, *w = nullptr, *z = nullptr, *xacc = nullptr, *rhs = nullptr, *sol = nullptr;
  double *hdev = nullptr, *partial = nullptr, *partial2 = nullptr;
  unsigned int* dot_counter = nullptr;
  TileGeom tg{};
  int *tile_ids = nullptr, *tile_count = nullptr, *tile_off = nullptr, *tile_cursor = nullptr;
  double* trec = nullptr;
  int* spos = nullptr;
  double* rs = nullptr;          // slip channel: blob and image positions (2M x 3) for spreading
  double* zsorted = nullptr;
  void* tabs = nullptr;          // spreading tables of the current configuration
  int *tab_start = nullptr, *tab_count = nullptr, *tab_order = nullptr;
  unsigned int* tab_claimed = nullptr;
  double* hhost = nullptr;   // pinned readback
  GmresState* gm = nullptr;  // device GMRES bookkeeping
  unsigned char* gm_host = nullptr;   // pinned: two status slots
  unsigned char* gm_host_dev = nullptr;   // the same memory as the device sees it
  hipEvent_t gm_ev[2] = {nullptr, nullptr};
  hipEvent_t step_ev[2] = {nullptr, nullptr};   // end of a step's update and readback, per slot

  // One HIP graph per Krylov column k of a GMRES iteration (preconditioner,
  // mobility apply, Arnoldi), captured the first time column k runs with a
  // given set of configuration arrays and replayed after; graphs = false
  // launches every kernel on its own.
  struct IterGraph {
    hipGraphExec_t exec = nullptr;
    const double *Y = nullptr, *q = nullptr, *r = nullptr;
  };
  std::vector<IterGraph> iter_graph;
  bool graphs = true;
  // The set-up of a step (noise, predictor, forces, tables, right-hand side,
  // |b|^2) captured once: its launches read the step from the device counter
  // step_dev, which the graph advances at its end; step_dev_val is the value
  // the counter holds for work queued next (UINT64_MAX: unknown).
  hipGraphExec_t setup_graph = nullptr;
  uint64_t* step_dev = nullptr;
  uint64_t step_dev_val = UINT64_MAX;
  // The end of a step (update and readback into slot k) captured once per slot.
  hipGraphExec_t done_graph[2] = {nullptr, nullptr};

  // Launches fused over suspensions (gdc_set_fusion): inside gdc_batch_step a
  // fused handle does not launch its GMRES iterations itself; the call
  // launches each iteration kernel once for all the handles that are ready
  // (fuse_live while such a call runs), on a stream of its own per group.
  // The two streams are joined only where work crosses: own_dirty says the
  // handle's stream holds work the fused stream has not waited for (join_ev
  // marks it); fuse_pending says the handle's stream has not yet waited for
  // its last fused iteration, whose end gm_ev[fuse_evslot] marks on fuse_on.
  bool fuse = false;
  bool fuse_live = false;
  hipEvent_t join_ev = nullptr;
  bool own_dirty = true;
  bool fuse_pending = false;
  int fuse_evslot = 0;
  hipStream_t fuse_on = nullptr;

  bool dry = false;               // footprint query: count device bytes, touch no device
  size_t dev_bytes = 0;           // device memory held by the handle
  bool has_state = false;         // Y, q hold a state (gdc_set_state or gdc_step)
  SolveRun sv;
  StepRun sr;
  std::vector<double> step_log;   // completion times of steps (ms, monotonic clock)
  // error counts of the steps completed since the last gdc_step / gdc_batch_step entry
  int n_overflow = 0, n_nonfinite = 0, n_notconv = 0, n_nonpos = 0;
  int n_fused = 0;   // GMRES iterations launched fused since the last reset_errors
  // sine forcing: the field (sin(k y), 0, 0) on the grid, its average at
  // each blob, f0/(eta k^2), and the amplitudes v_x of this call's steps
  void* grid_sine = nullptr;
  double* vbg = nullptr;
  double sine_scale = 0.0, sine_sum_coef = 0.0, sine_acc = 0.0;
  int sine_n = 0;
  // sums over the steps completed since reset_errors, for the call's means
  double its_acc = 0.0, nu_acc = 0.0, nu_acc2 = 0.0, nu_lo = 0.0, nu_hi = 0.0;
  int done_n = 0;

  ~gdc_handle() {
    for (IterGraph& g : iter_graph)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (setup_graph) (void)hipGraphExecDestroy(setup_graph);
    for (hipGraphExec_t g : done_graph)
      if (g) (void)hipGraphExecDestroy(g);
    for (void* p : allocs) (void)hipFree(p);
    if (hhost) (void)hipHostFree(hhost);
    if (gm_host) (void)hipHostFree(gm_host);
    for (hipEvent_t e : gm_ev)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : step_ev)
      if (e) (void)hipEventDestroy(e);
    if (join_ev) (void)hipEventDestroy(join_ev);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }

  template <typename T>
  int alloc(T** p, size_t count) {
    dev_bytes += std::max<size_t>(count, 1) * sizeof(T);
    if (dry) {
      *p = nullptr;
      return GDC_OK;
    }
    GDC_TRY(dalloc(p, count));
    allocs.push_back((void*)*p);
    return GDC_OK;
  }
};

namespace {

int validate(const gdc_config* c) {
  auto bad = [](const std::string& m) {
    set_error(m);
    return GDC_EINVAL;
  };
  if (!c) return bad("cfg is NULL");
  for (int d = 0; d < 3; ++d) {
    if (!(c->L[d] > 0.0)) return bad("L must be positive");
    if (c->n[d] % 2 != 0 || !fft_size_supported(c->n[d]))
      return bad("grid size must be even, 2^a 3^b and in [8, 384] (every such size the transforms take is parity-tested)");
  }
  if (!(c->a > 0.0) || c->sigma < 0.0 || c->trunc < 0.0) return bad("a must be > 0, sigma and trunc >= 0");
  if (!(c->eta > 0.0) || c->kT < 0.0 || !(c->dt > 0.0)) return bad("eta, dt must be > 0 and kT >= 0");
  if (c->fd_delta < 0.0 || c->gmres_tol < 0.0 || c->gmres_maxit < 0 || c->gmres_restart < 0)
    return bad("negative solver parameter");
  if (c->gmres_restart > 60) return bad("gmres_restart must be <= 60");
  if (c->precision != GDC_FP32 && c->precision != GDC_FP64) return bad("precision must be GDC_FP32 or GDC_FP64");
  if (c->scheme != GDC_SCHEME_GDC && c->scheme != GDC_SCHEME_EM) return bad("unknown scheme");
  if (c->divergence != GDC_DIV_FD && c->divergence != GDC_DIV_RFD) return bad("unknown divergence mode");
  if (c->n_shapes < 1 || !c->shapes) return bad("at least one shape is required");
  if (c->n_bodies < 1 || !c->body_shape) return bad("at least one body is required");
  long long M = 0;
  for (int s = 0; s < c->n_shapes; ++s)
    if (c->shapes[s].n_blobs < 1 || !c->shapes[s].b) return bad("every shape needs at least one blob");
  for (int p = 0; p < c->n_bodies; ++p) {
    if (c->body_shape[p] < 0 || c->body_shape[p] >= c->n_shapes) return bad("body_shape out of range");
    M += c->shapes[c->body_shape[p]].n_blobs;
  }
  if (M > (1LL << 30)) return bad("too many blobs");
  if (c->forces.steric_k < 0.0 || c->forces.steric_cutoff < 0.0) return bad("steric parameters must be >= 0");
  if (c->channel != 0 && c->channel != 1) return bad("channel must be 0 or 1");
  if (c->forces.wall_k < 0.0 || c->forces.wall_cutoff < 0.0) return bad("wall parameters must be >= 0");
  if (c->channel) {
    if (c->forces.shear_rate != 0.0 || c->forces.sine_force != 0.0)
      return bad("the slip channel takes no background shear or sine forcing");
    if (2 * M > (1LL << 30)) return bad("too many blobs");
  } else if (c->forces.wall_k > 0.0) {
    return bad("wall forces need the slip channel (channel = 1)");
  }
  return GDC_OK;
}

template <typename R>
const Cx<R>* const* tw_of(gdc_handle* h) {
  return reinterpret_cast<const Cx<R>* const*>(h->tw);
}

// Sorts the blobs at positions r by grid tile and builds the spreading
// tables; every spread at r needs them.
// zeroed: the tile counts and the table claim counter were cleared already
// (by the step's opening clear).
int prepare_positions(gdc_handle* h, const double* r, bool zeroed = false) {
  const double* rsp = r;
  if (h->geom.channel) {
    // the images of the slip channel are spread too (blobs M .. 2M - 1)
    GDC_TRY(mirror_positions(r, h->M, h->geom.L[1], h->rs, h->stream));
    rsp = h->rs;
  }
  GDC_TRY(tile_sort(h->geom, h->tg, rsp, h->Ms, h->tile_ids, h->tile_count, h->tile_off, h->tile_cursor, h->trec,
                    h->spos, h->stream, zeroed));
  if (h->precision == GDC_FP64)
    return spread_prepare<double>(h->geom, h->tg, h->trec, h->tile_off, h->tabs, h->tab_start, h->tab_count,
                                  h->tab_order, h->tab_claimed, h->stream, zeroed);
  return spread_prepare<float>(h->geom, h->tg, h->trec, h->tile_off, h->tabs, h->tab_start, h->tab_count,
                               h->tab_order, h->tab_claimed, h->stream, zeroed);
}

// The tile-sorted records averaging may visit blobs by (the real blobs only:
// in the slip channel the records also hold the images, so blobs are visited
// in index order instead; the sums are the same).
inline const void* sorted_records(const gdc_handle* h) { return h->geom.channel ? nullptr : h->trec; }

// out = M_FCM lam at blob positions r (prepared by prepare_positions), minus
// U_p + Omega_p x (r_i - Y_p) when V (N x 6) is given.
// Kernels launched with a non-null `skip` return at once when *skip != 0.
template <typename R>
int apply_mobility(gdc_handle* h, const double* r, const double* lam, double* out, const double* Y = nullptr,
                   const double* V = nullptr, const double* lam_sorted = nullptr, const int* skip = nullptr) {
  const GridGeom& g = h->geom;
  R* f = (R*)h->grid[0];
  GDC_TRY(spread<R>(g, h->tg, h->tabs, h->tab_order, lam, lam_sorted, f, h->stream, skip));
  GDC_TRY(stokes_solve<R>(g, tw_of<R>(h), f, (Cx<R>*)h->grid[1], (Cx<R>*)h->grid[2], h->stream, skip));
  return interp<R>(g, r, f, out, h->M, g.dV, h->bt.blob_body, Y, V, h->stream, skip, sorted_records(h));
}

// z = P^-1 x and y = A z, A = [[M, -K], [-K^T, -Pi]] at (Y, q, r).
template <typename R>
int apply_saddle_precond(gdc_handle* h, const double* Y, const double* q, const double* r, const double* x,
                         double* z, double* y, const int* skip = nullptr) {
  const long long m3 = 3LL * h->M;
  GDC_TRY(precond_apply(h->bt, q, x, z, y + m3, h->spos, h->zsorted, h->maxdim, h->stream, skip,
                        h->geom.channel ? h->M : 0));
  return apply_mobility<R>(h, r, z, y, Y, z + m3, h->zsorted, skip);
}

GmStatus read_status(const unsigned char* p) {
  GmStatus st;
  std::memcpy(&st.est, p, sizeof(double));
  std::memcpy(&st.its, p + 8, 4 * sizeof(int));
  return st;
}

// Queues a copy of the device status into pinned slot `slot` and an event
// after it.
int post_status_copy(gdc_handle* h, int slot) {
  GDC_HIP(hipMemcpyAsync(h->gm_host + 32 * slot, h->gm, GM_STATUS_BYTES, hipMemcpyDeviceToHost, h->stream));
  return GDC_OK;
}

int post_status(gdc_handle* h, int slot) {
  GDC_TRY(post_status_copy(h, slot));
  GDC_HIP(hipEventRecord(h->gm_ev[slot], h->stream));
  return GDC_OK;
}

// ready = whether event e has completed; waits for it when block is set.
int event_done(hipEvent_t e, bool block, bool& ready) {
  if (block) {
    GDC_HIP(hipEventSynchronize(e));
    ready = true;
    return GDC_OK;
  }
  const hipError_t q = hipEventQuery(e);
  if (q == hipErrorNotReady) {
    (void)hipGetLastError();   // "not ready" is an answer, not an error to carry
    ready = false;
    return GDC_OK;
  }
  if (q != hipSuccess) {
    set_error(std::string("hipEventQuery: ") + hipGetErrorString(q));
    return GDC_EDEVICE;
  }
  ready = true;
  return GDC_OK;
}

int poll_status(gdc_handle* h, int slot, bool block, bool& ready, GmStatus& st) {
  GDC_TRY(event_done(h->gm_ev[slot], block, ready));
  if (ready) st = read_status(h->gm_host + 32 * slot);
  return GDC_OK;
}

// Whether a GMRES iteration of h may be fused with other suspensions' now:
// inside gdc_batch_step, for a fused handle on the FP32 plane-path
// transforms with the matrix-core preconditioner, outside the slip channel
// and while no probe watches a kernel family.
bool fusable_now(const gdc_handle* h) {
  return h->fuse_live && !h->geom.channel && stokes_fusable(h->geom, h->precision) &&
         precond_fusable(h->bt, h->maxdim) && !probe_active();
}

// Queues GMRES iteration k of the current cycle: z = P^-1 V_k, w = A z (the
// mobility apply), and the Arnoldi step that writes V_{k+1}, the Hessenberg
// column and the status slot (k + 1) & 1.  With graphs on (and no kernel
// probe active) the launches of column k are captured once into a HIP graph
// and replayed on later cycles and steps: one launch instead of about ten.
// Every pointer the iteration uses is fixed for the handle except the
// configuration arrays (Y, q, r), which key the graph.
template <typename R>
int queue_iteration(gdc_handle* h, int k) {
  SolveRun& sv = h->sv;
  const long long n = h->nx;
  const int m = h->restart;
  hipStream_t s = h->stream;
  double* Vk = h->Vb + n * k;
  double* Vk1 = h->Vb + n * (k + 1);
  const int slot = (k + 1) & 1;
  auto enqueue = [&]() -> int {
    GDC_TRY(apply_saddle_precond<R>(h, sv.Y, sv.q, sv.r, Vk, h->z, h->w, &h->gm->done));
    return arnoldi_orthogonalise(h->w, h->Vb, n, k + 1, n, h->partial, h->partial2, Vk1, h->hdev,
                                 h->hdev + HCOLS, s, &h->gm->done, h->gm, m, h->gm_host_dev + 32 * slot);
  };
  if (!h->graphs || probe_active()) return enqueue();
  if ((int)h->iter_graph.size() < m) h->iter_graph.resize(m);
  gdc_handle::IterGraph& ig = h->iter_graph[k];
  if (!ig.exec || ig.Y != sv.Y || ig.q != sv.q || ig.r != sv.r) {
    if (ig.exec) {
      (void)hipGraphExecDestroy(ig.exec);
      ig.exec = nullptr;
    }
    GDC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    const int rc = enqueue();
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &graph);   // always leave capture mode
    if (rc != GDC_OK || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      if (rc != GDC_OK) return rc;
      set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      return GDC_EDEVICE;
    }
    const hipError_t e2 = hipGraphInstantiate(&ig.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) {
      ig.exec = nullptr;
      set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
      return GDC_EDEVICE;
    }
    ig.Y = sv.Y;
    ig.q = sv.q;
    ig.r = sv.r;
  }
  GDC_HIP(hipGraphLaunch(ig.exec, s));
  return GDC_OK;
}

// Right-preconditioned restarted GMRES (Saad & Schultz) on the saddle system
// with classical Gram-Schmidt and one reorthogonalisation, zero initial
// guess.  Solution (x = P^-1 u) written to h->sol.
//
// The Hessenberg bookkeeping runs on the device (in the last Arnoldi kernel,
// which also writes the status to pinned host memory), so the host
// queues iteration k + 1 before it reads the status of iteration k: the
// GPU never idles on the host.  When iteration k ends the cycle, the kernels
// already queued for iteration k + 1 see the device flag and return at once.
//
// solve_begin queues the set-up; each solve_advance queues the next piece of
// work or reads the next status (waiting for it when block is set, else
// reporting ADV_BLOCKED while it is not there yet) and reports ADV_DONE once
// h->sol is queued.
//
// The device part of solve_begin: |b|^2 and, in the same launch, the GMRES
// state; the solution accumulator is cleared by the first cycle's start.
int solve_begin_queue(gdc_handle* h) {
  const long long n = h->nx;
  return multi_dot(nullptr, n, 0, h->rhs, n, true, h->partial, h->dot_counter, h->hdev, h->stream, h->gm, h->tol,
                   h->maxit);
}

// The host part: the solve's resumable state.
void solve_begin_host(gdc_handle* h, const double* Y, const double* q, const double* r) {
  h->sv = SolveRun{};
  h->sv.Y = Y;
  h->sv.q = q;
  h->sv.r = r;
  h->sv.phase = SolveRun::CYCLE;
}

template <typename R>
int solve_begin(gdc_handle* h, const double* Y, const double* q, const double* r) {
  GDC_TRY(solve_begin_queue(h));
  solve_begin_host(h, Y, q, r);
  return GDC_OK;
}

template <typename R>
int solve_advance(gdc_handle* h, bool block, int& adv) {
  SolveRun& sv = h->sv;
  const long long n = h->nx;
  const int m = h->restart;
  hipStream_t s = h->stream;
  adv = ADV_PROGRESS;
  switch (sv.phase) {
    case SolveRun::CYCLE: {
      if (sv.first) {
        // zero initial guess: the residual is b, whose |b|^2 solve_begin
        // left in hdev[0]; V_0 = b / |b|
        GDC_TRY(scale_by_inv_sqrt(h->rhs, h->hdev, h->Vb, n, s, h->gm, h->xacc, n));
      } else {
        // w = b - A P^-1 xacc
        GDC_TRY(apply_saddle_precond<R>(h, sv.Y, sv.q, sv.r, h->xacc, h->z, h->w));
        GDC_TRY(sub_from(h->rhs, h->w, n, s));
        GDC_TRY(multi_dot(nullptr, n, 0, h->w, n, true, h->partial, h->dot_counter, h->hdev + 2 * HCOLS, s));
        GDC_TRY(scale_by_inv_sqrt(h->w, h->hdev + 2 * HCOLS, h->Vb, n, s, h->gm));
      }
      sv.first = false;
      GDC_TRY(post_status(h, 0));
      sv.k = 0;
      sv.queued = false;
      sv.phase = SolveRun::ITER;
      return GDC_OK;
    }
    case SolveRun::ITER: {
      const int k = sv.k;
      bool enq = false;
      if (sv.deferred) {   // waiting for the fused launch of this iteration
        adv = ADV_BLOCKED;
        return GDC_OK;
      }
      if (!sv.queued) {
        if (fusable_now(h)) {
          // gdc_batch_step launches it with the other ready suspensions and
          // then records gm_ev[(k + 1) & 1] on the fused launches' stream
          sv.queued = sv.deferred = true;
          adv = ADV_BLOCKED;
          return GDC_OK;
        }
        const int slot = (k + 1) & 1;
        GDC_TRY(queue_iteration<R>(h, k));
        GDC_HIP(hipEventRecord(h->gm_ev[slot], s));
        sv.queued = enq = true;
      }
      // status after iteration k - 1 (or after the cycle start)
      bool ready = false;
      GDC_TRY(poll_status(h, k & 1, block, ready, sv.st));
      if (!ready) {
        adv = enq ? ADV_PROGRESS : ADV_BLOCKED;
        return GDC_OK;
      }
      if (sv.st.done || k + 1 >= m) {
        sv.phase = SolveRun::FINISH;
      } else {
        sv.k = k + 1;
        sv.queued = false;
      }
      return GDC_OK;
    }
    case SolveRun::FINISH:
      GDC_TRY(gm_finish_cycle(h->gm, h->xacc, h->Vb, n, n, s));
      GDC_TRY(post_status(h, 0));
      sv.phase = SolveRun::FINISH_WAIT;
      return GDC_OK;
    case SolveRun::FINISH_WAIT: {
      bool ready = false;
      GDC_TRY(poll_status(h, 0, block, ready, sv.st));
      if (!ready) {
        adv = ADV_BLOCKED;
        return GDC_OK;
      }
      if (sv.st.converged || sv.st.its >= h->maxit) {
        GDC_TRY(precond_apply(h->bt, sv.q, h->xacc, h->sol, nullptr, nullptr, nullptr, h->maxdim, s));
        sv.res.its = sv.st.its;
        sv.res.relres = sv.st.est;
        sv.res.converged = sv.st.converged != 0;
        sv.phase = SolveRun::DONE;
        adv = ADV_DONE;
      } else {
        sv.phase = SolveRun::CYCLE;
      }
      return GDC_OK;
    }
    case SolveRun::DONE:
      adv = ADV_DONE;
      return GDC_OK;
    default:
      set_error("no solve in progress");
      return GDC_EINVAL;
  }
}

// The whole solve, waiting for each status.
template <typename R>
int gmres(gdc_handle* h, const double* Y, const double* q, const double* r, GmresResult& res) {
  GDC_TRY(solve_begin<R>(h, Y, q, r));
  int adv = ADV_PROGRESS;
  while (adv != ADV_DONE) GDC_TRY(solve_advance<R>(h, true, adv));
  res = h->sv.res;
  h->sv.phase = SolveRun::IDLE;
  return GDC_OK;
}

// Blob forces and body forces/torques at (Y, q, r) into h->F.
bool steric_on(const gdc_handle* h) {
  return h->cfg.forces.steric_k > 0.0 && h->cfg.forces.steric_cutoff > 0.0;
}

// zeroed: the pair-force cell counts were cleared already.
int forces_at(gdc_handle* h, const double* Y, const double* r, bool zeroed = false) {
  const gdc_forces& f = h->cfg.forces;
  const double* fb = nullptr;
  if (steric_on(h)) {
    GDC_TRY(steric_forces(h->bt, h->geom, r, f.steric_k, f.steric_cutoff, h->cell_count, h->cell_list,
                          h->cell_cap, h->nc, h->flags, h->fblob, h->stream, zeroed));
    fb = h->fblob;
  }
  if (h->geom.channel && f.wall_k > 0.0 && f.wall_cutoff > 0.0) {
    GDC_TRY(wall_forces(r, h->M, 0.5 * h->geom.L[1], f.wall_k, f.wall_cutoff, h->fblob, fb != nullptr, h->stream));
    fb = h->fblob;
  }
  return body_forces(h->bt, Y, r, fb, h->cforce, h->F, h->stream);
}

// Random velocity field of step `step` into h->grid_fl.
// step_ptr: the step is read from this device counter instead (captured set-up).
template <typename R>
int make_fluct(gdc_handle* h, uint64_t step, const uint64_t* step_ptr = nullptr) {
  const GridGeom& g = h->geom;
  if (h->cfg.kT == 0.0) return fill_zero(h->grid_fl, 3 * (size_t)g.G * sizeof(R), h->stream);
  return fluct_field<R>(g, tw_of<R>(h), (R*)h->grid_fl, (Cx<R>*)h->grid[1], (Cx<R>*)h->grid[2], h->cfg.seed,
                        step, h->cfg.kT, h->cfg.dt, h->stream, step_ptr);
}

// Steps 2-3 at the state in (h->Y, h->q): calV, d_p and nu on the device.
template <typename R>
int predictor_dev(gdc_handle* h, uint64_t step, const uint64_t* step_ptr = nullptr) {
  hipStream_t s = h->stream;
  const int mode = h->cfg.divergence == GDC_DIV_RFD ? 1 : 0;
  GDC_TRY(fd_displacements(h->bt, h->q, h->cfg.fd_delta, mode, h->cfg.seed, step, h->dr, h->wrfd, s, h->Y, h->r,
                           step_ptr));
  GDC_TRY(interp_fd<R>(h->geom, h->r, h->dr, mode == 1 ? 1 : 6, (const R*)h->grid_fl, h->v, h->vd, h->M, s));
  return body_lsq_div(h->bt, h->q, h->v, h->vd, h->wrfd, h->cfg.fd_delta, mode, h->calV, h->dp,
                      h->dot_counter + 1, 0.5 * h->cfg.dt, h->nu, s);
}

// Readback slot k of the pinned buffer: nu, the 4 error flags (2 doubles),
// the sine sum.
inline double* readback(gdc_handle* h, int k) { return h->hhost + 4 * HCOLS + 8 * k; }

// Takes in the readback of the oldest queued step: statistics, error counts,
// the step log.
void retire_step(gdc_handle* h, bool gdc_scheme) {
  StepRun& sr = h->sr;
  const double* rb = readback(h, sr.head);
  h->step_log.push_back(now_ms());
  sr.gr = sr.slot_gr[sr.head];
  sr.nu = gdc_scheme ? rb[0] : 1.0;
  const int* fl = reinterpret_cast<const int*>(rb + 1);
  if (fl[0]) ++h->n_overflow;
  if (fl[1]) ++h->n_nonfinite;
  if (!sr.gr.converged) ++h->n_notconv;
  if (!(sr.nu > 0.0)) ++h->n_nonpos;
  h->its_acc += sr.gr.its;
  h->nu_acc += sr.nu;
  h->nu_acc2 += sr.nu * sr.nu;
  h->nu_lo = h->done_n ? std::min(h->nu_lo, sr.nu) : sr.nu;
  h->nu_hi = h->done_n ? std::max(h->nu_hi, sr.nu) : sr.nu;
  ++h->done_n;
  if (h->vbg) {
    h->sine_acc += h->sine_scale + h->sine_sum_coef * rb[3];
    ++h->sine_n;
  }
  sr.head ^= 1;
  --sr.pend;
}

// Steps 1-5 of a step and the start of its solve, at the state (h->Y, h->q):
// the random field, the predictor and midpoint (or the blob positions), the
// forces, the tables of the midpoint configuration, the right-hand side and
// |b|^2.  The random numbers are those of `step`, or, with step_ptr, of the
// value in that device counter when the launches run.
template <typename R>
int enqueue_setup(gdc_handle* h, uint64_t step, const uint64_t* step_ptr, bool cycle_start) {
  hipStream_t s = h->stream;
  const bool gdc_scheme = h->cfg.scheme == GDC_SCHEME_GDC;
  // the step's counters in one launch: error flags, pair-force cell
  // counts, tile counts, spreading-table claim (none is read again before
  // this step uses it)
  {
    void* zp[4] = {h->flags, h->tile_count, h->tab_claimed, h->cell_count};
    const size_t zb[4] = {16, tile_count_bytes(h->tg), spread_claim_bytes(),
                          steric_on(h) ? cell_count_bytes(h->nc) : 0};
    GDC_TRY(fill_zero_many(zp, zb, 4, s));
  }
  GDC_TRY(make_fluct<R>(h, step, step_ptr));
  const double* Ym = h->Y;
  const double* qm = h->q;
  if (gdc_scheme) {
    GDC_TRY(predictor_dev<R>(h, step, step_ptr));
    GDC_TRY(midpoint_positions(h->bt, h->Y, h->q, h->calV, 0.5 * h->cfg.dt, h->Ym, h->qm, h->rm, s));
    Ym = h->Ym;
    qm = h->qm;
  } else {
    GDC_TRY(blob_positions(h->bt, Ym, qm, h->rm, s));
  }
  GDC_TRY(forces_at(h, Ym, h->rm, true));
  GDC_TRY(prepare_positions(h, h->rm, true));
  GDC_TRY(interp<R>(h->geom, h->rm, (const R*)h->grid_fl, h->v, h->M, h->geom.dV, nullptr, nullptr, nullptr, s,
                    nullptr, sorted_records(h)));
  if (h->vbg)
    GDC_TRY(interp<R>(h->geom, h->rm, (const R*)h->grid_sine, h->vbg, h->M, h->geom.dV, nullptr, nullptr,
                      nullptr, s, nullptr, sorted_records(h)));
  GDC_TRY(rhs_build(h->bt, qm, Ym, h->rm, h->v, h->vbg, h->sine_scale, h->F, h->cfg.forces.shear_rate,
                    h->geom.L[1], h->rhs, s));
  GDC_TRY(solve_begin_queue(h));
  if (!cycle_start) return GDC_OK;
  // the first cycle's start, as solve_advance queues it (V_0 = b / |b|, its
  // status into slot 0; the caller records the status event)
  const long long n = h->nx;
  GDC_TRY(scale_by_inv_sqrt(h->rhs, h->hdev, h->Vb, n, s, h->gm, h->xacc, n));
  return post_status_copy(h, 0);
}

// Queues the set-up of step `step`.  With graphs on (and no kernel probe
// active) its launches are captured once into a HIP graph, with the step
// read from the handle's device counter, which the graph then advances; a
// replay is one launch (two when the counter has to be set first, after
// gdc_set_step or steps taken without the graph).  Every pointer the set-up
// uses is fixed for the handle.
template <typename R>
int queue_setup(gdc_handle* h, uint64_t step, bool& cycle_started) {
  hipStream_t s = h->stream;
  cycle_started = false;
  if (!h->graphs || probe_active()) return enqueue_setup<R>(h, step, nullptr, false);
  if (!h->setup_graph) {
    GDC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    int rc = enqueue_setup<R>(h, step, h->step_dev, true);
    if (rc == GDC_OK) rc = step_counter_bump(h->step_dev, s);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &graph);   // always leave capture mode
    if (rc != GDC_OK || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      if (rc != GDC_OK) return rc;
      set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      return GDC_EDEVICE;
    }
    const hipError_t e2 = hipGraphInstantiate(&h->setup_graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) {
      h->setup_graph = nullptr;
      set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
      return GDC_EDEVICE;
    }
  }
  if (h->step_dev_val != step) GDC_TRY(step_counter_set(h->step_dev, step, s));
  GDC_HIP(hipGraphLaunch(h->setup_graph, s));
  h->step_dev_val = step + 1;
  cycle_started = true;
  return GDC_OK;
}

// Queues the end of a step into readback slot k: the sine sum (forced
// rheology), the update (step 6) and the copies of nu and the error flags.
// With graphs on (and no probe) it is captured once per slot.
int queue_step_end(gdc_handle* h, int k) {
  hipStream_t s = h->stream;
  const bool gdc_scheme = h->cfg.scheme == GDC_SCHEME_GDC;
  double* rb = readback(h, k);
  auto enqueue = [&]() -> int {
    if (h->vbg) {
      // sum_i lambda_ix J[sin(k y)](r_i) of the midpoint solve, for v_x
      GDC_TRY(blob_dot_x(h->sol, h->vbg, h->M, h->nu + 1, s));
      GDC_HIP(hipMemcpyAsync(rb + 3, h->nu + 1, sizeof(double), hipMemcpyDeviceToHost, s));
    }
    GDC_TRY(update(h->bt, h->Y, h->q, h->sol + 3LL * h->M, gdc_scheme ? h->nu : nullptr, h->cfg.dt,
                   h->flags + 1, s));
    GDC_HIP(hipMemcpyAsync(rb, h->nu, sizeof(double), hipMemcpyDeviceToHost, s));
    GDC_HIP(hipMemcpyAsync(rb + 1, h->flags, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
    return GDC_OK;
  };
  if (!h->graphs || probe_active()) return enqueue();
  hipGraphExec_t& ge = h->done_graph[k];
  if (!ge) {
    GDC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    const int rc = enqueue();
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &graph);   // always leave capture mode
    if (rc != GDC_OK || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      if (rc != GDC_OK) return rc;
      set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      return GDC_EDEVICE;
    }
    const hipError_t e2 = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) {
      ge = nullptr;
      set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
      return GDC_EDEVICE;
    }
  }
  GDC_HIP(hipGraphLaunch(ge, s));
  return GDC_OK;
}

// Time steps of the resident state (h->Y, h->q) as a resumable, pipelined
// run.  Each advance does one thing:
//   - retires the oldest queued step whose readback has landed (ADV_DONE);
//   - IDLE, with steps left to start: queues the noise, steps 2-4, the
//     forces and the right-hand side and starts the solve;
//   - SOLVE: advances the solve; when it is done, queues the update (step 6)
//     and the readback into the next free slot and returns to IDLE, so the
//     following step is queued behind it at once.
// With block set and nothing else to do it waits for the oldest readback
// or for the solve's next status.
template <typename R>
int step_advance(gdc_handle* h, bool block, int& adv) {
  hipStream_t s = h->stream;
  StepRun& sr = h->sr;
  const bool gdc_scheme = h->cfg.scheme == GDC_SCHEME_GDC;
  adv = ADV_PROGRESS;
  if (sr.pend > 0) {
    bool ready = false;
    GDC_TRY(event_done(h->step_ev[sr.head], false, ready));
    if (ready) {
      retire_step(h, gdc_scheme);
      adv = ADV_DONE;
      return GDC_OK;
    }
  }
  if (sr.phase == StepRun::IDLE && sr.to_start > 0 && sr.pend < 2) {
    const uint64_t step = h->step;
    const double* Ym = gdc_scheme ? h->Ym : h->Y;
    const double* qm = gdc_scheme ? h->qm : h->q;
    bool cycle_started = false;
    GDC_TRY(queue_setup<R>(h, step, cycle_started));
    solve_begin_host(h, Ym, qm, h->rm);
    if (cycle_started) {
      // the captured set-up also started the first GMRES cycle
      GDC_HIP(hipEventRecord(h->gm_ev[0], s));
      h->sv.first = false;
      h->sv.k = 0;
      h->sv.queued = false;
      h->sv.phase = SolveRun::ITER;
    }
    --sr.to_start;
    sr.phase = StepRun::SOLVE;
    return GDC_OK;
  }
  if (sr.phase == StepRun::SOLVE) {
    int a = ADV_PROGRESS;
    // the oldest readback lands before any status of this solve, so a
    // blocking wait goes to it first
    GDC_TRY(solve_advance<R>(h, block && sr.pend == 0, a));
    if (a == ADV_DONE) {
      const int k = (sr.head + sr.pend) & 1;
      sr.slot_gr[k] = h->sv.res;
      h->sv.phase = SolveRun::IDLE;
      GDC_TRY(queue_step_end(h, k));
      GDC_HIP(hipEventRecord(h->step_ev[k], s));
      ++sr.pend;
      h->step += 1;   // the next step draws the next noise
      sr.phase = StepRun::IDLE;
      return GDC_OK;
    }
    if (a == ADV_PROGRESS) return GDC_OK;
  }
  if (block && sr.pend > 0) {
    bool ready = false;
    GDC_TRY(event_done(h->step_ev[sr.head], true, ready));
    retire_step(h, gdc_scheme);
    adv = ADV_DONE;
    return GDC_OK;
  }
  adv = ADV_BLOCKED;
  return GDC_OK;
}

int step_advance_any(gdc_handle* h, bool block, int& adv) {
  return h->precision == GDC_FP64 ? step_advance<double>(h, block, adv) : step_advance<float>(h, block, adv);
}

// Return code for the errors counted since the last reset_errors.
int step_errors(const gdc_handle* h) {
  if (h->n_overflow) {
    set_error("pair-force cell list overflow");
    return GDC_ENUMERIC;
  }
  if (h->n_nonfinite) {
    set_error("non-finite positions or orientations");
    return GDC_ENUMERIC;
  }
  if (h->n_notconv) {
    set_error("GMRES did not reach the tolerance in at least one step");
    return GDC_ENOTCONV;
  }
  return GDC_OK;
}

void reset_errors(gdc_handle* h) {
  h->n_overflow = h->n_nonfinite = h->n_notconv = h->n_nonpos = 0;
  h->n_fused = 0;
  h->sine_acc = 0.0;
  h->sine_n = 0;
  h->its_acc = h->nu_acc = h->nu_acc2 = h->nu_lo = h->nu_hi = 0.0;
  h->done_n = 0;
}

double sine_mean(const gdc_handle* h) { return h->sine_n ? h->sine_acc / h->sine_n : 0.0; }

// Statistics of the steps completed since reset_errors (the last step's
// solve, the call's means).
void fill_stats(const gdc_handle* h, gdc_stats* st) {
  st->gmres_iterations = h->sr.gr.its;
  st->gmres_relres = h->sr.gr.relres;
  st->nu = h->sr.nu;
  st->nu_nonpositive = h->n_nonpos;
  st->sine_vx = sine_mean(h);
  st->gmres_iterations_mean = h->done_n ? h->its_acc / h->done_n : 0.0;
  st->nu_mean = h->done_n ? h->nu_acc / h->done_n : 0.0;
  st->nu_std = h->done_n ? std::sqrt(std::max(0.0, h->nu_acc2 / h->done_n - st->nu_mean * st->nu_mean)) : 0.0;
  st->nu_min = h->nu_lo;
  st->nu_max = h->nu_hi;
  st->status = step_errors(h);
  st->fused_iterations = h->n_fused;
}

int require_idle(const gdc_handle* h) {
  if (h->sr.phase != StepRun::IDLE || h->sv.phase != SolveRun::IDLE || h->sr.pend != 0) {
    set_error("the handle has a step in flight: finish it with gdc_batch_step first");
    return GDC_EINVAL;
  }
  return GDC_OK;
}

int copy_in(gdc_handle* h, double* dst, const double* src, size_t count, int memspace) {
  const hipMemcpyKind kind = memspace == GDC_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  GDC_HIP(hipMemcpyAsync(dst, src, count * sizeof(double), kind, h->stream));
  return GDC_OK;
}

int copy_out(gdc_handle* h, double* dst, const double* src, size_t count, int memspace) {
  const hipMemcpyKind kind = memspace == GDC_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  GDC_HIP(hipMemcpyAsync(dst, src, count * sizeof(double), kind, h->stream));
  return GDC_OK;
}

int check_quaternions(const gdc_handle* h, const double* Y, const double* q) {
  for (long long k = 0; k < 3LL * h->N; ++k)
    if (!std::isfinite(Y[k])) {
      set_error("non-finite position of body " + std::to_string(k / 3));
      return GDC_EINVAL;
    }
  for (int p = 0; p < h->N; ++p) {
    const double* qp = q + 4LL * p;
    const double nrm = std::sqrt(qp[0] * qp[0] + qp[1] * qp[1] + qp[2] * qp[2] + qp[3] * qp[3]);
    if (!(std::fabs(nrm - 1.0) <= 1e-6)) {
      set_error("quaternion " + std::to_string(p) + " is not of unit norm");
      return GDC_EINVAL;
    }
  }
  return GDC_OK;
}

// Host arrays are checked on the host before anything is copied.  Device
// arrays are copied into the midpoint buffers (free between steps), checked
// there by a kernel whose flags the host reads back, and only then become
// the state: a rejected state leaves the handle's state as it was.
int load_state(gdc_handle* h, const double* Y, const double* q, int memspace) {
  if (!Y || !q) {
    set_error("Y and q are required");
    return GDC_EINVAL;
  }
  if (memspace != GDC_HOST && memspace != GDC_DEVICE) {
    set_error("memspace must be GDC_HOST or GDC_DEVICE");
    return GDC_EINVAL;
  }
  if (memspace == GDC_HOST) {
    GDC_TRY(check_quaternions(h, Y, q));
    GDC_TRY(copy_in(h, h->Y, Y, 3 * (size_t)h->N, memspace));
    return copy_in(h, h->q, q, 4 * (size_t)h->N, memspace);
  }
  GDC_TRY(copy_in(h, h->Ym, Y, 3 * (size_t)h->N, memspace));
  GDC_TRY(copy_in(h, h->qm, q, 4 * (size_t)h->N, memspace));
  GDC_TRY(fill_zero(h->flags, 16, h->stream));
  GDC_TRY(check_state(h->Ym, h->qm, h->N, 1e-6, h->flags + 2, h->stream));
  int* fl = reinterpret_cast<int*>(h->hhost + 4 * HCOLS + 16);
  GDC_HIP(hipMemcpyAsync(fl, h->flags + 2, 2 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
  GDC_HIP(hipStreamSynchronize(h->stream));
  if (fl[0]) {
    set_error("non-finite position in the device array Y");
    return GDC_EINVAL;
  }
  if (fl[1]) {
    set_error("a quaternion of the device array q is not of unit norm");
    return GDC_EINVAL;
  }
  GDC_TRY(copy_in(h, h->Y, h->Ym, 3 * (size_t)h->N, GDC_DEVICE));
  return copy_in(h, h->q, h->qm, 4 * (size_t)h->N, GDC_DEVICE);
}

int finish(gdc_handle* h) {
  GDC_HIP(hipStreamSynchronize(h->stream));
  return GDC_OK;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int d) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(d);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

template <typename R>
int init_grid_tables(gdc_handle* h) {
  for (int d = 0; d < 3; ++d) {
    const int n = h->geom.n[d];
    std::vector<Cx<R>> t(n);
    for (int k = 0; k < n; ++k) {
      const long double ang = 2.0L * 3.141592653589793238462643383279503L * (long double)k / (long double)n;
      t[k] = Cx<R>{(R)std::cos(ang), (R)(-std::sin(ang))};
    }
    Cx<R>* dptr = nullptr;
    GDC_TRY(h->alloc(&dptr, n));
    if (!h->dry) {
      GDC_HIP(hipMemcpyAsync(dptr, t.data(), n * sizeof(Cx<R>), hipMemcpyHostToDevice, h->stream));
      GDC_HIP(hipStreamSynchronize(h->stream));
    }
    h->tw[d] = dptr;
  }
  // The three work fields are one allocation, so grid[1] and grid[2] together
  // also hold a 3 x G FP64 field.
  R* base = nullptr;
  GDC_TRY(h->alloc(&base, 9 * (size_t)h->geom.G));
  for (int k = 0; k < 3; ++k) h->grid[k] = base + 3 * (size_t)h->geom.G * k;
  R* p = nullptr;
  GDC_TRY(h->alloc(&p, 3 * (size_t)h->geom.G));
  h->grid_fl = p;
  return GDC_OK;
}

int init_impl(const gdc_config* cfg, gdc_handle* h) {
  GDC_TRY(validate(cfg));
  h->cfg = *cfg;
  h->cfg.shapes = nullptr;
  h->cfg.body_shape = nullptr;
  gdc_config& c = h->cfg;
  if (c.sigma == 0.0) c.sigma = c.a / std::sqrt(3.14159265358979323846);
  if (c.trunc == 0.0) c.trunc = 3.0 * c.a;
  if (c.fd_delta == 0.0) c.fd_delta = 1e-6;
  if (c.gmres_tol == 0.0) c.gmres_tol = 1e-6;
  if (c.gmres_maxit == 0) c.gmres_maxit = 200;
  if (c.gmres_restart == 0) c.gmres_restart = 50;
  h->tol = c.gmres_tol;
  h->maxit = c.gmres_maxit;
  h->restart = c.gmres_restart;
  h->precision = c.precision;
  h->rsize = c.precision == GDC_FP64 ? 8 : 4;
  h->device = c.device;

  GridGeom& g = h->geom;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = c.n[d];
    g.L[d] = c.L[d];
    g.dx[d] = c.L[d] / c.n[d];
    g.inv_dx[d] = 1.0 / g.dx[d];
    if (!(2.0 * c.trunc < c.L[d])) {
      set_error("the envelope cutoff must be below half the box length");
      return GDC_EINVAL;
    }
    g.P[d] = (int)std::floor(2.0 * c.trunc / g.dx[d]) + 1;
  }
  if (g.P[2] > 58) {   // averaging keeps a blob's axis-2 factors in 64 entries
    set_error("the envelope spans " + std::to_string(g.P[2]) + " grid points along axis 2; at most 58 are supported");
    return GDC_EINVAL;
  }
  g.n2h = g.n[2] / 2;
  g.G = (long long)g.n[0] * g.n[1] * g.n[2];
  g.dV = g.dx[0] * g.dx[1] * g.dx[2];
  g.eta = c.eta;
  g.sigma = c.sigma;
  g.rc = c.trunc;
  g.rc2 = c.trunc * c.trunc;
  g.inv2s2 = 1.0 / (2.0 * c.sigma * c.sigma);
  g.wnorm = std::pow(2.0 * 3.14159265358979323846 * c.sigma * c.sigma, -1.5);
  g.tiled = (g.n[0] % 8 == 0 && g.n[1] % 8 == 0 && g.n[2] % 32 == 0) ? 1 : 0;
  g.channel = c.channel;

  // shapes and bodies
  h->N = cfg->n_bodies;
  h->shapes.resize(cfg->n_shapes);
  std::vector<double> shape_b;
  std::vector<int> shape_boff(cfg->n_shapes + 1, 0);
  std::vector<double> pinv(36 * cfg->n_shapes), nul(36 * cfg->n_shapes), Lp(cfg->n_shapes);
  std::vector<double> precT;
  std::vector<long long> prec_off(cfg->n_shapes);
  for (int s = 0; s < cfg->n_shapes; ++s) {
    ShapeHost& S = h->shapes[s];
    S.nb = cfg->shapes[s].n_blobs;
    S.b.assign(cfg->shapes[s].b, cfg->shapes[s].b + 3 * S.nb);
    std::string err;
    if (!build_shape(S, c.a, c.eta, err)) {
      set_error("shape " + std::to_string(s) + ": " + err);
      return GDC_EINVAL;
    }
    shape_boff[s + 1] = shape_boff[s] + S.nb;
    shape_b.insert(shape_b.end(), S.b.begin(), S.b.end());
    std::memcpy(&pinv[36 * s], S.pinv, sizeof(S.pinv));
    std::memcpy(&nul[36 * s], S.null, sizeof(S.null));
    Lp[s] = S.Lp;
    prec_off[s] = (long long)precT.size();
    precT.insert(precT.end(), S.precT.begin(), S.precT.end());
    h->maxdim = std::max(h->maxdim, 3 * S.nb + 6);
  }
  h->body_shape.assign(cfg->body_shape, cfg->body_shape + h->N);
  std::vector<int> body_off(h->N + 1, 0);
  for (int p = 0; p < h->N; ++p) body_off[p + 1] = body_off[p] + h->shapes[h->body_shape[p]].nb;
  h->M = body_off[h->N];
  std::vector<int> blob_body(h->M), blob_local(h->M);
  for (int p = 0; p < h->N; ++p)
    for (int k = 0; k < body_off[p + 1] - body_off[p]; ++k) {
      blob_body[body_off[p] + k] = p;
      blob_local[body_off[p] + k] = k;
    }
  h->nx = 3LL * h->M + 6LL * h->N;
  h->Ms = h->M * (c.channel ? 2 : 1);

  // device (a footprint query touches none)
  if (!h->dry) {
    int ndev = 0;
    GDC_HIP(hipGetDeviceCount(&ndev));
    if (c.device < 0 || c.device >= ndev) {
      set_error("device ordinal out of range");
      return GDC_EINVAL;
    }
    GDC_HIP(hipSetDevice(c.device));
    {
      void* sp = nullptr;
      GDC_TRY(scratch_address(c.device, &sp));
    }
    if (c.stream) {
      h->stream = (hipStream_t)c.stream;
    } else {
      // non-blocking: work of other handles and the legacy stream does not
      // serialise with this handle's
      GDC_HIP(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
      h->own_stream = true;
    }
  }

  auto upload = [&](auto** dst, const auto& vec) -> int {
    using T = typename std::remove_reference<decltype(vec)>::type::value_type;
    T* p = nullptr;
    GDC_TRY(h->alloc(&p, vec.size()));
    if (!h->dry && !vec.empty())
      GDC_HIP(hipMemcpyAsync(p, vec.data(), vec.size() * sizeof(T), hipMemcpyHostToDevice, h->stream));
    *dst = p;
    return GDC_OK;
  };
  BodyTables& B = h->bt;
  B.N = h->N;
  B.M = h->M;
  B.n_shapes = cfg->n_shapes;
  int *d_bs, *d_boff, *d_bb, *d_bl, *d_sboff;
  double *d_sb, *d_pinv, *d_null, *d_Lp, *d_prec;
  long long* d_poff;
  GDC_TRY(upload(&d_bs, h->body_shape));
  GDC_TRY(upload(&d_boff, body_off));
  GDC_TRY(upload(&d_bb, blob_body));
  GDC_TRY(upload(&d_bl, blob_local));
  GDC_TRY(upload(&d_sb, shape_b));
  GDC_TRY(upload(&d_sboff, shape_boff));
  GDC_TRY(upload(&d_pinv, pinv));
  GDC_TRY(upload(&d_null, nul));
  GDC_TRY(upload(&d_Lp, Lp));
  GDC_TRY(upload(&d_prec, precT));
  GDC_TRY(upload(&d_poff, prec_off));
  B.body_shape = d_bs;
  B.body_off = d_boff;
  B.blob_body = d_bb;
  B.blob_local = d_bl;
  B.shape_b = d_sb;
  B.shape_boff = d_sboff;
  B.shape_pinv = d_pinv;
  B.shape_null = d_null;
  B.shape_Lp = d_Lp;
  B.shape_precT = d_prec;
  B.shape_prec_off = d_poff;
  {
    // bodies grouped by shape for the matrix-core preconditioner: as many
    // per group (4, 8 or 16, the columns of one MFMA tile) as leave at least
    // PREC_MIN_GROUPS groups, so that large suspensions stage each shape
    // block for 16 bodies and small ones keep enough workgroups to hide the
    // gather latency.  A body's result does not depend on its group.
    int grp = PREC_GROUP_MIN;
    while (2 * grp <= PREC_GROUP_MAX && (long long)h->N >= (long long)PREC_MIN_GROUPS * 2 * grp) grp *= 2;
    std::vector<int> gbody, gfirst, gcount, gshape;
    for (int sh = 0; sh < cfg->n_shapes; ++sh) {
      const int first = (int)gbody.size();
      for (int p = 0; p < h->N; ++p)
        if (h->body_shape[p] == sh) gbody.push_back(p);
      for (int k = first; k < (int)gbody.size(); k += grp) {
        gfirst.push_back(k);
        gcount.push_back(std::min(grp, (int)gbody.size() - k));
        gshape.push_back(sh);
      }
    }
    int *d_gb, *d_gf, *d_gc, *d_gs;
    GDC_TRY(upload(&d_gb, gbody));
    GDC_TRY(upload(&d_gf, gfirst));
    GDC_TRY(upload(&d_gc, gcount));
    GDC_TRY(upload(&d_gs, gshape));
    B.n_groups = (int)gfirst.size();
    B.group_body = d_gb;
    B.group_first = d_gf;
    B.group_count = d_gc;
    B.group_shape = d_gs;
    B.mfma = h->maxdim <= PREC_MFMA_MAXDIM ? 1 : 0;
  }

  const size_t N = h->N, M = h->M;
  GDC_TRY(h->alloc(&h->Y, 3 * N));
  GDC_TRY(h->alloc(&h->q, 4 * N));
  GDC_TRY(h->alloc(&h->Ym, 3 * N));
  GDC_TRY(h->alloc(&h->qm, 4 * N));
  GDC_TRY(h->alloc(&h->r, 3 * M));
  GDC_TRY(h->alloc(&h->rm, 3 * M));
  GDC_TRY(h->alloc(&h->v, 3 * M));
  GDC_TRY(h->alloc(&h->vd, 18 * M));
  GDC_TRY(h->alloc(&h->dr, 18 * M));
  GDC_TRY(h->alloc(&h->wrfd, 6 * N));
  GDC_TRY(h->alloc(&h->calV, 6 * N));
  GDC_TRY(h->alloc(&h->dp, N));
  GDC_TRY(h->alloc(&h->nu, 2));
  GDC_TRY(h->alloc(&h->F, 6 * N));
  GDC_TRY(h->alloc(&h->fblob, 3 * M));
  GDC_TRY(h->alloc(&h->flags, 4));
  GDC_TRY(h->alloc(&h->io, std::max(6 * N, 3 * M)));
  std::vector<double> cf(c.forces.const_force, c.forces.const_force + 6);
  GDC_TRY(upload(&h->cforce, cf));
  if (!h->dry) GDC_HIP(hipMemsetAsync(h->flags, 0, 4 * sizeof(int), h->stream));

  const gdc_forces& f = c.forces;
  if (f.steric_k > 0.0 && f.steric_cutoff > 0.0) {
    long long ncell = 1;
    for (int d = 0; d < 3; ++d) {
      h->nc[d] = (int)std::floor(c.L[d] / f.steric_cutoff);
      if (h->nc[d] < 3) {
        set_error("the box must span at least three pair-force cells per axis");
        return GDC_EINVAL;
      }
      ncell *= h->nc[d];
    }
    h->cell_cap = 32;
    GDC_TRY(h->alloc(&h->cell_count, (size_t)((ncell * 4 + 15) / 16 * 4)));
    GDC_TRY(h->alloc(&h->cell_list, (size_t)(ncell * h->cell_cap)));
  }

  const size_t nx = (size_t)h->nx;
  GDC_TRY(h->alloc(&h->Vb, (size_t)(h->restart + 1) * nx));
  GDC_TRY(h->alloc(&h->w, nx));
  GDC_TRY(h->alloc(&h->z, nx));
  GDC_TRY(h->alloc(&h->xacc, nx + 2));
  GDC_TRY(h->alloc(&h->rhs, nx));
  GDC_TRY(h->alloc(&h->sol, nx + 2));
  GDC_TRY(h->alloc(&h->hdev, 5 * HCOLS));
  GDC_TRY(h->alloc(&h->partial, std::max((size_t)DOT_MAX_BLOCKS, (size_t)(h->nx / 1024 + 1)) * HCOLS));
  GDC_TRY(h->alloc(&h->partial2, std::max((size_t)DOT_MAX_BLOCKS, (size_t)(h->nx / 1024 + 1)) * HCOLS));
  GDC_TRY(h->alloc(&h->dot_counter, 4));
  if (!h->dry) GDC_HIP(hipMemsetAsync(h->dot_counter, 0, 4 * sizeof(unsigned int), h->stream));
  {
    TileGeom& t = h->tg;
    const int Tdef[3] = {8, 8, 32};
    t.ntiles = 1;
    for (int d = 0; d < 3; ++d) {
      t.T[d] = std::min(Tdef[d], g.n[d]);
      t.nt[d] = (g.n[d] + t.T[d] - 1) / t.T[d];
      const int reach = (int)std::ceil(c.trunc / g.dx[d]) + 1;
      t.H[d] = (reach + t.T[d] - 1) / t.T[d];
      if (t.H[d] > 2) {
        set_error("the envelope cutoff spans too many grid points for the spreading tiles");
        return GDC_EINVAL;
      }
      t.ntiles *= t.nt[d];
    }
    t.wz8 = (g.P[2] <= 8 && t.nt[2] >= 2) ? 1 : 0;
    const int cols = std::min(t.T[1], g.P[1]) * std::min(t.T[2], g.P[2]);
    t.S = 1;
    while (t.S < cols) t.S *= 2;
    const size_t Ms = (size_t)h->Ms;
    GDC_TRY(h->alloc(&h->tile_ids, Ms));
    GDC_TRY(h->alloc(&h->trec, 2 * Ms * tile_record_bytes() / sizeof(double)));
    GDC_TRY(h->alloc(&h->spos, Ms));
    GDC_TRY(h->alloc(&h->zsorted, 3 * Ms));
    if (c.channel) GDC_TRY(h->alloc(&h->rs, 3 * Ms));
    GDC_TRY(h->alloc(&h->tile_count, (size_t)(t.ntiles + 4)));
    GDC_TRY(h->alloc(&h->tile_off, (size_t)(t.ntiles + 1)));
    GDC_TRY(h->alloc(&h->tile_cursor, (size_t)t.ntiles));
    {
      double* tabs = nullptr;
      GDC_TRY(h->alloc(&tabs, (spread_table_bytes(g, t, h->Ms, h->precision) + 7) / 8));
      h->tabs = tabs;
    }
    GDC_TRY(h->alloc(&h->tab_start, (size_t)t.ntiles));
    GDC_TRY(h->alloc(&h->tab_count, (size_t)t.ntiles));
    GDC_TRY(h->alloc(&h->tab_order, 4 * (size_t)t.ntiles));
    GDC_TRY(h->alloc(&h->tab_claimed, spread_claim_bytes() / sizeof(unsigned int)));
  }
  GDC_TRY(h->alloc(&h->gm, 1));
  GDC_TRY(h->alloc(&h->step_dev, 2));
  if (!h->dry) {
    GDC_HIP(hipHostMalloc((void**)&h->hhost, 5 * HCOLS * sizeof(double), hipHostMallocDefault));
    GDC_HIP(hipHostMalloc((void**)&h->gm_host, 64, hipHostMallocMapped | hipHostMallocCoherent));
    GDC_HIP(hipHostGetDevicePointer((void**)&h->gm_host_dev, h->gm_host, 0));
    for (hipEvent_t& e : h->gm_ev) GDC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (hipEvent_t& e : h->step_ev) GDC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    GDC_HIP(hipEventCreateWithFlags(&h->join_ev, hipEventDisableTiming));
  }

  if (h->precision == GDC_FP64) {
    GDC_TRY(init_grid_tables<double>(h));
  } else {
    GDC_TRY(init_grid_tables<float>(h));
  }
  if (c.forces.sine_force != 0.0) {
    const double k = 2.0 * 3.14159265358979323846 / g.L[1];
    h->sine_scale = c.forces.sine_force / (c.eta * k * k);
    h->sine_sum_coef = 2.0 / (g.L[0] * g.L[1] * g.L[2]) / (c.eta * k * k);
    GDC_TRY(h->alloc(&h->vbg, 3 * (size_t)h->M));
    if (h->precision == GDC_FP64) {
      double* f = nullptr;
      GDC_TRY(h->alloc(&f, 3 * (size_t)g.G));
      if (!h->dry) GDC_TRY(fill_sine_field<double>(g, f, h->stream));
      h->grid_sine = f;
    } else {
      float* f = nullptr;
      GDC_TRY(h->alloc(&f, 3 * (size_t)g.G));
      if (!h->dry) GDC_TRY(fill_sine_field<float>(g, f, h->stream));
      h->grid_sine = f;
    }
  }
  // the host vectors of the uploads above go out of scope on return
  if (!h->dry) GDC_HIP(hipStreamSynchronize(h->stream));
  if (!h->dry) {
    if (h->precision == GDC_FP64) {
      GDC_TRY(fft_autotune<double>(h->geom, tw_of<double>(h), (double*)h->grid[0], (Cx<double>*)h->grid[1],
                                   (Cx<double>*)h->grid[2], h->stream));
    } else {
      GDC_TRY(fft_autotune<float>(h->geom, tw_of<float>(h), (float*)h->grid[0], (Cx<float>*)h->grid[1],
                                  (Cx<float>*)h->grid[2], h->stream));
    }
    GDC_HIP(hipStreamSynchronize(h->stream));
  }
  return GDC_OK;
}

}  // namespace

extern "C" {

const char* gdc_last_error(void) { return gdc::g_last_error.c_str(); }

int gdc_init(const gdc_config* cfg, gdc_handle** out) {
  if (!out) {
    set_error("out is NULL");
    return GDC_EINVAL;
  }
  *out = nullptr;
  gdc_handle* h = new (std::nothrow) gdc_handle();
  if (!h) {
    set_error("host allocation failed");
    return GDC_ENOMEM;
  }
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  const int rc = init_impl(cfg, h);
  if (rc != GDC_OK) {
    delete h;
    if (prev >= 0) (void)hipSetDevice(prev);
    return rc;
  }
  if (prev >= 0) (void)hipSetDevice(prev);
  *out = h;
  return GDC_OK;
}

void gdc_free(gdc_handle* h) {
  if (!h) return;
  DeviceGuard dg(h->device);
  (void)hipStreamSynchronize(h->stream);
  delete h;
}

int gdc_mobility_apply(gdc_handle* h, int mode, const double* Y, const double* q, const double* in, double* out,
                       int memspace) {
  if (!h || !in || !out) {
    set_error("handle, in and out are required");
    return GDC_EINVAL;
  }
  if (mode != GDC_BLOB && mode != GDC_BODY) {
    set_error("mode must be GDC_BLOB or GDC_BODY");
    return GDC_EINVAL;
  }
  DeviceGuard dg(h->device);
  hipStream_t s = h->stream;
  GDC_TRY(require_idle(h));
  GDC_TRY(load_state(h, Y, q, memspace));
  GDC_TRY(blob_positions(h->bt, h->Y, h->q, h->r, s));
  GDC_TRY(fill_zero(h->flags, 16, s));
  GmresResult gr;
  gr.converged = true;
  if (mode == GDC_BLOB) {
    GDC_TRY(copy_in(h, h->io, in, 3 * (size_t)h->M, memspace));
    GDC_TRY(prepare_positions(h, h->r));
    // in the slip channel spreading reads the forces (and their images) in
    // the sorted order
    const double* lsort = nullptr;
    if (h->geom.channel) {
      GDC_TRY(sort_forces(h->io, h->spos, h->M, h->M, h->zsorted, s));
      lsort = h->zsorted;
    }
    if (h->precision == GDC_FP64) {
      GDC_TRY(apply_mobility<double>(h, h->r, h->io, h->v, nullptr, nullptr, lsort));
    } else {
      GDC_TRY(apply_mobility<float>(h, h->r, h->io, h->v, nullptr, nullptr, lsort));
    }
    GDC_TRY(check_finite(h->v, 3LL * h->M, h->flags + 1, s));
    GDC_TRY(copy_out(h, out, h->v, 3 * (size_t)h->M, memspace));
  } else {
    GDC_TRY(copy_in(h, h->io, in, 6 * (size_t)h->N, memspace));
    GDC_TRY(rhs_build(h->bt, h->q, h->Y, h->r, nullptr, nullptr, 0.0, h->io, 0.0, h->geom.L[1], h->rhs, s));
    GDC_TRY(prepare_positions(h, h->r));
    if (h->precision == GDC_FP64) {
      GDC_TRY(gmres<double>(h, h->Y, h->q, h->r, gr));
    } else {
      GDC_TRY(gmres<float>(h, h->Y, h->q, h->r, gr));
    }
    GDC_TRY(check_finite(h->sol + 3LL * h->M, 6LL * h->N, h->flags + 1, s));
    GDC_TRY(copy_out(h, out, h->sol + 3LL * h->M, 6 * (size_t)h->N, memspace));
  }
  GDC_HIP(hipMemcpyAsync(h->hhost, h->flags, 4 * sizeof(int), hipMemcpyDeviceToHost, s));
  GDC_TRY(finish(h));
  const int* fl = reinterpret_cast<const int*>(h->hhost);
  if (fl[1]) {
    set_error("non-finite mobility result");
    return GDC_ENUMERIC;
  }
  if (!gr.converged) {
    set_error("GMRES did not reach the tolerance (relative residual " + std::to_string(gr.relres) + ")");
    return GDC_ENOTCONV;
  }
  return GDC_OK;
}

int gdc_step(gdc_handle* h, int n_steps, double* Y, double* q, int memspace, gdc_stats* st) {
  if (!h || n_steps < 0) {
    set_error("a handle and n_steps >= 0 are required");
    return GDC_EINVAL;
  }
  DeviceGuard dg(h->device);
  GDC_TRY(require_idle(h));
  const auto t0 = std::chrono::steady_clock::now();
  GDC_TRY(load_state(h, Y, q, memspace));
  h->has_state = true;
  reset_errors(h);
  h->sr.to_start = n_steps;
  for (int done = 0; done < n_steps;) {
    int adv = ADV_PROGRESS;
    GDC_TRY(step_advance_any(h, true, adv));
    if (adv == ADV_DONE) ++done;
    if (adv == ADV_BLOCKED) {
      set_error("step pipeline stalled");
      return GDC_EINVAL;
    }
  }
  GDC_TRY(copy_out(h, Y, h->Y, 3 * (size_t)h->N, memspace));
  GDC_TRY(copy_out(h, q, h->q, 4 * (size_t)h->N, memspace));
  GDC_TRY(finish(h));
  if (st) {
    st->steps_done = n_steps;
    fill_stats(h, st);
    st->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  return step_errors(h);
}

int gdc_set_state(gdc_handle* h, const double* Y, const double* q, int memspace) {
  if (!h) {
    set_error("handle is required");
    return GDC_EINVAL;
  }
  DeviceGuard dg(h->device);
  GDC_TRY(require_idle(h));
  GDC_TRY(load_state(h, Y, q, memspace));
  GDC_TRY(finish(h));
  h->has_state = true;
  h->step_log.clear();
  h->step_log.push_back(now_ms());
  return GDC_OK;
}

int gdc_get_state(gdc_handle* h, double* Y, double* q, int memspace) {
  if (!h || !Y || !q || (memspace != GDC_HOST && memspace != GDC_DEVICE)) {
    set_error("handle, Y, q and a valid memspace are required");
    return GDC_EINVAL;
  }
  DeviceGuard dg(h->device);
  GDC_TRY(require_idle(h));
  if (!h->has_state) {
    set_error("the handle holds no state: call gdc_set_state or gdc_step first");
    return GDC_EINVAL;
  }
  GDC_TRY(copy_out(h, Y, h->Y, 3 * (size_t)h->N, memspace));
  GDC_TRY(copy_out(h, q, h->q, 4 * (size_t)h->N, memspace));
  return finish(h);
}

namespace {

// Staging of fused launches.  Each group of handles that share every kernel
// instantiation (its key) launches on a stream of its own, one of up to
// FUSE_STREAMS per GPU, so the groups of different grid sizes overlap.  The
// argument tables go from a pinned host slot to a device slot in one copy
// on that stream; a stream's slots are used in turn, and a slot is reused
// only once its event (recorded after the launches that read it) has
// completed.
using FuseKey = std::array<int, 8>;
struct FuseSlot {
  void* host = nullptr;
  void* dev = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool used = false;
};
struct FuseStream {
  hipStream_t stream = nullptr;
  std::vector<FuseSlot> slots;
  int next = 0;
};
struct FuseDevice {
  std::vector<FuseStream> streams;
  std::map<FuseKey, int> of_key;
};
std::mutex g_fuse_mutex;
std::map<int, FuseDevice> g_fuse;
constexpr int FUSE_STREAMS = 4;
constexpr int FUSE_SLOTS = 8;

// The stream of group `key` on `device` (the current device) and its next
// staging slot, with room for `bytes`.
int fuse_slot(int device, const FuseKey& key, size_t bytes, FuseStream*& fst, FuseSlot*& slot) {
  FuseDevice& fd = g_fuse[device];
  auto it = fd.of_key.find(key);
  int si;
  if (it != fd.of_key.end()) {
    si = it->second;
  } else {
    si = (int)(fd.of_key.size() % FUSE_STREAMS);
    fd.of_key[key] = si;
  }
  if ((int)fd.streams.size() <= si) fd.streams.resize(si + 1);
  fst = &fd.streams[si];
  if (!fst->stream) {
    GDC_HIP(hipStreamCreateWithFlags(&fst->stream, hipStreamNonBlocking));
    fst->slots.resize(FUSE_SLOTS);
  }
  slot = &fst->slots[fst->next];
  fst->next = (fst->next + 1) % FUSE_SLOTS;
  if (slot->used) GDC_HIP(hipEventSynchronize(slot->ev));   // its launches are long done in practice
  if (!slot->ev) GDC_HIP(hipEventCreateWithFlags(&slot->ev, hipEventDisableTiming));
  if (slot->cap < bytes) {
    if (slot->host) GDC_HIP(hipHostFree(slot->host));
    if (slot->dev) GDC_HIP(hipFree(slot->dev));
    slot->host = slot->dev = nullptr;
    slot->cap = 0;
    const size_t cap = std::max<size_t>(bytes, 64 << 10);
    GDC_HIP(hipHostMalloc(&slot->host, cap, hipHostMallocDefault));
    GDC_HIP(hipMalloc(&slot->dev, cap));
    slot->cap = cap;
  }
  return GDC_OK;
}

// Whether the handle's next advance queues nothing on its own stream: inside
// a GMRES cycle it only defers its next iteration to a fused launch or polls
// the status of one.
bool fused_only(const gdc_handle* h) {
  return h->sr.phase == StepRun::SOLVE && h->sv.phase == SolveRun::ITER && fusable_now(h);
}

// Whether group `key` already has two fused iterations in flight on its
// stream: its ready handles then wait for the next pass, so that more of the
// group's handles join the launch while the GPU still has work queued.
bool fuse_busy(int device, const FuseKey& key) {
  std::lock_guard<std::mutex> lk(g_fuse_mutex);
  auto d = g_fuse.find(device);
  if (d == g_fuse.end()) return false;
  auto it = d->second.of_key.find(key);
  if (it == d->second.of_key.end() || it->second >= (int)d->second.streams.size()) return false;
  const FuseStream& fst = d->second.streams[it->second];
  int pending = 0;
  for (int back = 1; back <= 2; ++back) {
    const FuseSlot& sl = fst.slots[(fst.next + FUSE_SLOTS - back) % FUSE_SLOTS];
    if (!sl.used) continue;
    const hipError_t q = hipEventQuery(sl.ev);
    if (q == hipErrorNotReady) {
      (void)hipGetLastError();
      ++pending;
    }
  }
  return pending >= 2;
}

// The handle's stream waits for its last fused iteration (before the handle
// queues work of its own there).
int join_fused(gdc_handle* h) {
  if (!h->fuse_pending) return GDC_OK;
  GDC_HIP(hipStreamWaitEvent(h->stream, h->gm_ev[h->fuse_evslot], 0));
  h->fuse_pending = false;
  return GDC_OK;
}

// Byte layout of one fused iteration's tables: per kernel an argument array
// (ns entries) and the first block of every suspension (ns ints; for
// spreading, one table per spreading-table width).
struct FuseLayout {
  size_t pre, spr, fwd, prj, inv, itp, arn;            // argument arrays
  size_t f_pre, f_spr, f_pl, f_prj, f_itp, f_dot, f_axp, f_fin;   // first-block arrays
  size_t bytes;
  explicit FuseLayout(int ns) {
    size_t o = 0;
    auto take = [&](size_t b) {
      const size_t at = o;
      o = (o + b + 255) & ~size_t(255);
      return at;
    };
    pre = take(ns * sizeof(PrecondArgs));
    spr = take(ns * sizeof(SpreadArgs));
    fwd = take(ns * sizeof(PlaneArgs));
    prj = take(ns * sizeof(ProjPlaneArgs));
    inv = take(ns * sizeof(PlaneArgs));
    itp = take(ns * sizeof(InterpArgs));
    arn = take(ns * sizeof(ArnoldiArgs));
    f_pre = take(ns * sizeof(int));
    f_spr = take(ns * sizeof(int));
    f_pl = take(ns * sizeof(int));
    f_prj = take(ns * sizeof(int));
    f_itp = take(ns * sizeof(int));
    f_dot = take(ns * sizeof(int));
    f_axp = take(ns * sizeof(int));
    f_fin = take(ns * sizeof(int));
    bytes = o;
  }
};

int blocks_of(const LocalGrid& g) { return g.gx * g.gy * g.gz; }

// One fused GMRES iteration for handles that can share every kernel
// instantiation but spreading's (same grid, workgroup sizes and
// vector-length class), each at its own Krylov column: the same arithmetic,
// per suspension, as queue_iteration.  g lists the handles with 8-wide
// spreading tables first; spreading is launched once per table width.
int fuse_group(const FuseKey& key, const std::vector<gdc_handle*>& g) {
  const int ns = (int)g.size();
  const FuseLayout L(ns);
  std::lock_guard<std::mutex> lk(g_fuse_mutex);
  FuseStream* fst = nullptr;
  FuseSlot* slot = nullptr;
  GDC_TRY(fuse_slot(g[0]->device, key, L.bytes, fst, slot));
  unsigned char* hb = (unsigned char*)slot->host;
  unsigned char* db = (unsigned char*)slot->dev;
  auto* pa = (PrecondArgs*)(hb + L.pre);
  auto* sa = (SpreadArgs*)(hb + L.spr);
  auto* fa = (PlaneArgs*)(hb + L.fwd);
  auto* qa = (ProjPlaneArgs*)(hb + L.prj);
  auto* ia = (PlaneArgs*)(hb + L.inv);
  auto* ta = (InterpArgs*)(hb + L.itp);
  auto* aa = (ArnoldiArgs*)(hb + L.arn);
  int* f_pre = (int*)(hb + L.f_pre);
  int* f_spr = (int*)(hb + L.f_spr);
  int* f_pl = (int*)(hb + L.f_pl);
  int* f_prj = (int*)(hb + L.f_prj);
  int* f_itp = (int*)(hb + L.f_itp);
  int* f_dot = (int*)(hb + L.f_dot);
  int* f_axp = (int*)(hb + L.f_axp);
  int* f_fin = (int*)(hb + L.f_fin);
  int t_pre = 0, t_pl = 0, t_prj = 0, t_itp = 0, t_dot = 0, t_axp = 0, t_fin = 0;
  int n8 = 0, t_spr[2] = {0, 0};   // spreading: handles with 8-wide tables, blocks per width
  for (int j = 0; j < ns; ++j) {
    gdc_handle* h = g[j];
    SolveRun& sv = h->sv;
    const long long n = h->nx;
    const int k = sv.k;
    const long long m3 = 3LL * h->M;
    double* Vk = h->Vb + n * k;
    double* Vk1 = h->Vb + n * (k + 1);
    const int* skip = &h->gm->done;
    precond_describe(pa[j], h->bt, sv.q, Vk, h->z, h->w + m3, h->spos, h->zsorted, skip, 0);
    spread_describe(sa[j], h->geom, h->tg, h->tabs, h->tab_order, h->z, h->zsorted, h->grid[0], skip);
    StokesArgs st;
    stokes_describe(st, h->geom, (const void* const*)h->tw, h->grid[0], h->grid[1], skip);
    fa[j] = st.fwd;
    qa[j] = st.proj;
    ia[j] = st.inv;
    interp_describe(ta[j], h->geom, sv.r, h->grid[0], h->w, h->M, h->geom.dV, h->bt.blob_body, sv.Y, h->z + m3,
                    skip, sorted_records(h));
    GDC_TRY(arnoldi_describe(aa[j], h->w, h->Vb, n, k + 1, n, h->partial, h->partial2, Vk1, h->hdev,
                             h->hdev + HCOLS, skip, h->gm, h->restart, h->gm_host_dev + 32 * ((k + 1) & 1)));
    f_pre[j] = t_pre;
    t_pre += blocks_of(pa[j].grid);
    const int w = h->tg.wz8 ? 0 : 1;
    if (w == 0) ++n8;
    f_spr[j] = t_spr[w];
    t_spr[w] += blocks_of(sa[j].grid);
    f_pl[j] = t_pl;
    t_pl += blocks_of(fa[j].grid);
    f_prj[j] = t_prj;
    t_prj += blocks_of(qa[j].grid);
    f_itp[j] = t_itp;
    t_itp += blocks_of(ta[j].grid);
    f_dot[j] = t_dot;
    t_dot += blocks_of(aa[j].g_dot);
    f_axp[j] = t_axp;
    t_axp += blocks_of(aa[j].g_axpy);
    f_fin[j] = t_fin;
    t_fin += blocks_of(aa[j].g_fin);
  }
  hipStream_t fs = fst->stream;
  // the fused launches follow what each handle queued on its own stream
  // since the last join, and its previous fused iteration
  for (gdc_handle* h : g) {
    if (h->own_dirty) {
      GDC_HIP(hipEventRecord(h->join_ev, h->stream));
      GDC_HIP(hipStreamWaitEvent(fs, h->join_ev, 0));
      h->own_dirty = false;
    }
    if (h->fuse_pending && h->fuse_on != fs) GDC_HIP(hipStreamWaitEvent(fs, h->gm_ev[h->fuse_evslot], 0));
  }
  GDC_HIP(hipMemcpyAsync(db, hb, L.bytes, hipMemcpyHostToDevice, fs));
  const int* df_spr = (const int*)(db + L.f_spr);
  const auto* dsa = (const SpreadArgs*)(db + L.spr);
  GDC_TRY(precond_fused((const PrecondArgs*)(db + L.pre), ns, (const int*)(db + L.f_pre), t_pre, fs));
  GDC_TRY(spread_fused<float>(dsa, n8, 1, df_spr, t_spr[0], fs));
  GDC_TRY(spread_fused<float>(dsa + n8, ns - n8, 0, df_spr + n8, t_spr[1], fs));
  GDC_TRY(stokes_fused(g[0]->geom, (const PlaneArgs*)(db + L.fwd), (const ProjPlaneArgs*)(db + L.prj),
                       (const PlaneArgs*)(db + L.inv), ns, (const int*)(db + L.f_pl), t_pl,
                       (const int*)(db + L.f_prj), t_prj, fs));
  GDC_TRY(interp_fused<float>((const InterpArgs*)(db + L.itp), ns, (const int*)(db + L.f_itp), t_itp, fs));
  GDC_TRY(arnoldi_fused((const ArnoldiArgs*)(db + L.arn), ns, aa[0].shortv, (const int*)(db + L.f_dot), t_dot,
                        (const int*)(db + L.f_axp), t_axp, (const int*)(db + L.f_fin), t_fin, fs));
  GDC_HIP(hipEventRecord(slot->ev, fs));
  slot->used = true;
  // gm_ev marks the iteration's status, as solve_advance expects, on the
  // fused stream; the handle's own stream waits for it only before the
  // handle's next work of its own (join_fused)
  for (gdc_handle* h : g) {
    const int st = (h->sv.k + 1) & 1;
    GDC_HIP(hipEventRecord(h->gm_ev[st], fs));
    h->fuse_pending = true;
    h->fuse_evslot = st;
    h->fuse_on = fs;
    h->sv.deferred = false;
    ++h->n_fused;
  }
  return GDC_OK;
}

// Launches the deferred iterations of hs: one fused launch per kernel for
// each group of handles that share every kernel instantiation but
// spreading's; with hold set, not for a group with two fused iterations in
// flight.  Returns the number of handles launched in `launched`.
int fuse_flush(gdc_handle* const* hs, int nh, int& launched, bool hold) {
  launched = 0;
  std::map<FuseKey, std::vector<gdc_handle*>> groups;
  for (int i = 0; i < nh; ++i) {
    gdc_handle* h = hs[i];
    if (!h->sv.deferred) continue;
    const FftShape& f = h->geom.fft;
    const int shortv = h->nx <= (long long)DOT_MAX_BLOCKS * 256 ? 1 : 0;
    groups[{h->device, h->geom.n[0], h->geom.n[1], h->geom.n[2], f.plane_fwd, f.proj_plane, f.plane_inv, shortv}]
        .push_back(h);
  }
  int cur = -1;
  for (auto& kv : groups) {
    if (kv.first[0] != cur) {
      GDC_HIP(hipSetDevice(kv.first[0]));
      cur = kv.first[0];
    }
    if (hold && fuse_busy(kv.first[0], kv.first)) continue;
    std::vector<gdc_handle*>& g = kv.second;
    std::stable_partition(g.begin(), g.end(), [](const gdc_handle* h) { return h->tg.wz8 != 0; });
    GDC_TRY(fuse_group(kv.first, g));
    launched += (int)g.size();
  }
  return GDC_OK;
}

}  // namespace

int gdc_set_fusion(gdc_handle* h, int on) {
  if (!h) {
    set_error("handle is required");
    return GDC_EINVAL;
  }
  GDC_TRY(require_idle(h));
  h->fuse = on != 0;
  return GDC_OK;
}

int gdc_get_fusion(const gdc_handle* h, int* on) {
  if (!h || !on) {
    set_error("handle and output are required");
    return GDC_EINVAL;
  }
  *on = h->fuse ? 1 : 0;
  return GDC_OK;
}

int gdc_batch_step(gdc_handle* const* hs, int nh, int* steps, int until, double max_ms, gdc_stats* st) {
  if (nh < 0 || (nh > 0 && (!hs || !steps)) || (until != GDC_UNTIL_ALL && until != GDC_UNTIL_ANY) ||
      !(max_ms >= 0.0)) {
    set_error("gdc_batch_step: bad arguments");
    return GDC_EINVAL;
  }
  for (int i = 0; i < nh; ++i) {
    if (!hs[i] || steps[i] < 0) {
      set_error("gdc_batch_step: handle " + std::to_string(i) + " is NULL or has a negative step count");
      return GDC_EINVAL;
    }
    if (!hs[i]->has_state) {
      set_error("gdc_batch_step: handle " + std::to_string(i) + " holds no state (gdc_set_state)");
      return GDC_EINVAL;
    }
    // steps already queued by an earlier call count towards steps[i]
    const int inflight = (hs[i]->sr.phase == StepRun::SOLVE ? 1 : 0) + hs[i]->sr.pend;
    if (steps[i] < inflight) {
      set_error("gdc_batch_step: handle " + std::to_string(i) + " has " + std::to_string(inflight) +
                " steps in flight but only " + std::to_string(steps[i]) + " left");
      return GDC_EINVAL;
    }
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) {
        set_error("gdc_batch_step: a handle appears twice");
        return GDC_EINVAL;
      }
  }
  int prev_dev = -1;
  if (hipGetDevice(&prev_dev) != hipSuccess) prev_dev = -1;
  const double t0 = now_ms();
  // failed: the handle's state went non-finite (or its pair-force cell list
  // overflowed) in this call; it is not advanced further
  std::vector<int> watched(nh, 0), done_here(nh, 0), failed(nh, 0);
  std::vector<double> t_last(nh, 0.0);
  bool any_watched = false;
  for (int i = 0; i < nh; ++i) {
    watched[i] = steps[i] > 0;
    any_watched = any_watched || watched[i];
    hs[i]->sr.to_start = steps[i] - (hs[i]->sr.phase == StepRun::SOLVE ? 1 : 0) - hs[i]->sr.pend;
    reset_errors(hs[i]);
    hs[i]->fuse_live = hs[i]->fuse;
    hs[i]->own_dirty = true;
  }
  int rc = GDC_OK;
  int cur_dev = -1;
  while (any_watched) {
    bool progressed = false;
    for (int i = 0; i < nh && rc == GDC_OK; ++i) {
      gdc_handle* h = hs[i];
      if (steps[i] == 0 || failed[i]) continue;
      if (h->device != cur_dev) {
        if (hipSetDevice(h->device) != hipSuccess) {
          set_error("hipSetDevice failed");
          rc = GDC_EDEVICE;
          break;
        }
        cur_dev = h->device;
      }
      // queue all the work this handle can take before it must wait
      while (steps[i] > 0) {
        int adv = ADV_BLOCKED;
        if (!fused_only(h)) {
          // this advance may queue work on the handle's own stream
          const int r = join_fused(h);
          if (r != GDC_OK) {
            rc = r;
            break;
          }
          h->own_dirty = true;
        }
        const int r = step_advance_any(h, false, adv);
        if (r != GDC_OK) {
          set_error("gdc_batch_step: handle " + std::to_string(i) + ": " + gdc_last_error());
          rc = r;
          break;
        }
        if (adv == ADV_BLOCKED) break;
        progressed = true;
        if (adv == ADV_DONE) {
          --steps[i];
          ++done_here[i];
          t_last[i] = h->step_log.back() - t0;
          if (h->n_nonfinite || h->n_overflow) {
            failed[i] = 1;
            break;
          }
        }
      }
    }
    if (rc == GDC_OK) {
      // the iterations the fused handles deferred in this pass
      int launched = 0;
      const int r = fuse_flush(hs, nh, launched, true);
      if (r != GDC_OK) {
        set_error(std::string("gdc_batch_step: fused launch: ") + gdc_last_error());
        rc = r;
      }
      if (launched) {
        progressed = true;
        cur_dev = -1;
      }
    }
    if (rc != GDC_OK) break;
    bool all_zero = true, any_hit = false;
    for (int i = 0; i < nh; ++i) {
      all_zero = all_zero && (steps[i] == 0 || failed[i]);
      any_hit = any_hit || (watched[i] && (steps[i] == 0 || failed[i]));
    }
    if (all_zero || (until == GDC_UNTIL_ANY && any_hit)) break;
    if (max_ms > 0.0 && now_ms() - t0 >= max_ms) break;
    if (!progressed) std::this_thread::yield();
  }
  for (int i = 0; i < nh; ++i) {
    hs[i]->fuse_live = false;
    // an error between a deferral and its launch leaves nothing half-queued
    if (hs[i]->sv.deferred) {
      hs[i]->sv.deferred = false;
      hs[i]->sv.queued = false;
    }
    // later calls find all of the handle's work behind its own stream
    if (hs[i]->device != cur_dev && hipSetDevice(hs[i]->device) == hipSuccess) cur_dev = hs[i]->device;
    const int r = join_fused(hs[i]);
    if (r != GDC_OK && rc == GDC_OK) rc = r;
  }
  if (prev_dev >= 0) (void)hipSetDevice(prev_dev);
  // every handle's own outcome first; the message names the first failing
  // handle (or keeps the call's own error)
  const std::string call_error = rc != GDC_OK ? gdc_last_error() : std::string();
  int first_err = GDC_OK;
  std::string first_msg;
  for (int i = 0; i < nh; ++i) {
    gdc_handle* h = hs[i];
    const int e = step_errors(h);
    if (e != GDC_OK && first_err == GDC_OK) {
      first_err = e;
      first_msg = "handle " + std::to_string(i) + ": " + gdc_last_error();
    }
    if (st) {
      st[i].steps_done = done_here[i];
      fill_stats(h, &st[i]);
      st[i].ms = t_last[i];
    }
  }
  if (rc != GDC_OK) {
    set_error(call_error);
    return rc;
  }
  set_error(first_msg);
  return first_err;
}

int gdc_step_log(gdc_handle* h, double* t_ms, int cap, int* count) {
  if (!h || !count || cap < 0 || (cap > 0 && !t_ms)) {
    set_error("handle, count and a buffer of cap entries are required");
    return GDC_EINVAL;
  }
  const int n = (int)std::min<size_t>((size_t)cap, h->step_log.size());
  if (n > 0) std::memcpy(t_ms, h->step_log.data(), n * sizeof(double));
  *count = n;
  // the last entry stays: the next step's latency is measured from it
  if (!h->step_log.empty()) {
    const double last = h->step_log.back();
    if ((size_t)n == h->step_log.size()) {
      h->step_log.assign(1, last);
    } else {
      h->step_log.erase(h->step_log.begin(), h->step_log.begin() + n);
    }
  }
  return GDC_OK;
}

int gdc_footprint(const gdc_config* cfg, size_t* bytes) {
  if (!bytes) {
    set_error("bytes is NULL");
    return GDC_EINVAL;
  }
  *bytes = 0;
  std::unique_ptr<gdc_handle> h(new (std::nothrow) gdc_handle());
  if (!h) {
    set_error("host allocation failed");
    return GDC_ENOMEM;
  }
  h->dry = true;
  GDC_TRY(init_impl(cfg, h.get()));
  *bytes = h->dev_bytes;
  return GDC_OK;
}

int gdc_device_bytes(const gdc_handle* h, size_t* bytes) {
  if (!h || !bytes) {
    set_error("handle and bytes are required");
    return GDC_EINVAL;
  }
  *bytes = h->dev_bytes;
  return GDC_OK;
}

int gdc_probe_kernel(const char* family) {
  for (hipEvent_t e : g_probe.ev) (void)hipEventDestroy(e);
  g_probe = Probe{};
  if (!family || !family[0]) return GDC_OK;
  g_probe.ev.resize(2 * PROBE_PAIRS);
  for (auto& e : g_probe.ev) GDC_HIP(hipEventCreate(&e));
  g_probe.family = family;
  return GDC_OK;
}

int gdc_probe_read(double* total_ms, long long* launches, float* each_ms, long long capacity) {
  if (!total_ms || !launches || (each_ms && capacity < 0)) {
    set_error("outputs are required (and capacity >= 0 with each_ms)");
    return GDC_EINVAL;
  }
  double tot = 0.0;
  long long n = 0;
  for (size_t k = 0; k + 1 < g_probe.used; k += 2) {
    GDC_HIP(hipEventSynchronize(g_probe.ev[k + 1]));
    float ms = 0.f;
    GDC_HIP(hipEventElapsedTime(&ms, g_probe.ev[k], g_probe.ev[k + 1]));
    if (each_ms && n < capacity) each_ms[n] = ms;
    tot += ms;
    ++n;
  }
  *total_ms = tot;
  *launches = n;
  g_probe.used = 0;
  return GDC_OK;
}

int gdc_get_launch_config(const gdc_handle* h, int* threads, int n) {
  if (!h || !threads || n < GDC_FFT_PASSES) {
    set_error("handle and GDC_FFT_PASSES outputs are required");
    return GDC_EINVAL;
  }
  const FftShape& f = h->geom.fft;
  const int v[GDC_FFT_PASSES] = {f.plane_fwd, f.proj_plane, f.plane_inv, f.r2c, f.fwd1, f.proj, f.inv1, f.c2r};
  for (int k = 0; k < GDC_FFT_PASSES; ++k) threads[k] = v[k];
  return GDC_OK;
}

int gdc_set_launch_config(gdc_handle* h, const int* threads, int n) {
  if (!h || !threads || n < GDC_FFT_PASSES) {
    set_error("handle and GDC_FFT_PASSES sizes are required");
    return GDC_EINVAL;
  }
  GDC_TRY(require_idle(h));
  for (int k = 0; k < GDC_FFT_PASSES; ++k) {
    const int t = threads[k];
    const bool plane = k == 0 || k == 2;
    if (!(t == 256 || t == 512 || (plane && t == 1024))) {
      set_error("FFT workgroup size " + std::to_string(t) + " not allowed for pass " + std::to_string(k));
      return GDC_EINVAL;
    }
  }
  // captured iterations and set-ups hold the old kernels
  for (gdc_handle::IterGraph& g : h->iter_graph)
    if (g.exec) {
      (void)hipGraphExecDestroy(g.exec);
      g.exec = nullptr;
    }
  if (h->setup_graph) {
    (void)hipGraphExecDestroy(h->setup_graph);
    h->setup_graph = nullptr;
  }
  FftShape& f = h->geom.fft;
  f.plane_fwd = threads[0];
  f.proj_plane = threads[1];
  f.plane_inv = threads[2];
  f.r2c = threads[3];
  f.fwd1 = threads[4];
  f.proj = threads[5];
  f.inv1 = threads[6];
  f.c2r = threads[7];
  return GDC_OK;
}

int gdc_set_graphs(gdc_handle* h, int on) {
  if (!h) {
    set_error("handle is required");
    return GDC_EINVAL;
  }
  GDC_TRY(require_idle(h));
  h->graphs = on != 0;
  return GDC_OK;
}

int gdc_get_graphs(const gdc_handle* h, int* on) {
  if (!h || !on) {
    set_error("handle and output are required");
    return GDC_EINVAL;
  }
  *on = h->graphs ? 1 : 0;
  return GDC_OK;
}

int gdc_get_step(const gdc_handle* h, uint64_t* step) {
  if (!h || !step) {
    set_error("handle and step are required");
    return GDC_EINVAL;
  }
  *step = h->step;
  return GDC_OK;
}

int gdc_set_step(gdc_handle* h, uint64_t step) {
  if (!h) {
    set_error("handle is required");
    return GDC_EINVAL;
  }
  GDC_TRY(require_idle(h));
  h->step = step;
  return GDC_OK;
}

int gdc_fluct_velocity(gdc_handle* h, uint64_t step, double* u, int memspace) {
  if (!h || !u) {
    set_error("handle and output are required");
    return GDC_EINVAL;
  }
  DeviceGuard dg(h->device);
  GDC_TRY(require_idle(h));
  const size_t n = 3 * (size_t)h->geom.G;
  if (h->precision == GDC_FP64) {
    GDC_TRY(make_fluct<double>(h, step));
    if (h->geom.tiled) {
      // row-major copy in the (free) first two work fields, then out
      double* tmp = (double*)h->grid[1];
      GDC_TRY(field_to_rowmajor(h->geom, (const double*)h->grid_fl, tmp, h->stream));
      GDC_TRY(copy_out(h, u, tmp, n, memspace));
    } else {
      GDC_TRY(copy_out(h, u, (const double*)h->grid_fl, n, memspace));
    }
  } else {
    GDC_TRY(make_fluct<float>(h, step));
    // widen into the (free) first grid buffer pair, row-major, then copy out
    double* tmp = (double*)h->grid[1];
    GDC_TRY(field_to_rowmajor(h->geom, (const float*)h->grid_fl, tmp, h->stream));
    GDC_TRY(copy_out(h, u, tmp, n, memspace));
  }
  return finish(h);
}

int gdc_predictor(gdc_handle* h, const double* Y, const double* q, uint64_t step, double* calV, double* d,
                  int memspace) {
  if (!h || !calV || !d) {
    set_error("handle and outputs are required");
    return GDC_EINVAL;
  }
  DeviceGuard dg(h->device);
  GDC_TRY(require_idle(h));
  GDC_TRY(load_state(h, Y, q, memspace));
  if (h->precision == GDC_FP64) {
    GDC_TRY(make_fluct<double>(h, step));
    GDC_TRY(predictor_dev<double>(h, step));
  } else {
    GDC_TRY(make_fluct<float>(h, step));
    GDC_TRY(predictor_dev<float>(h, step));
  }
  GDC_TRY(copy_out(h, calV, h->calV, 6 * (size_t)h->N, memspace));
  GDC_TRY(copy_out(h, d, h->dp, (size_t)h->N, memspace));
  return finish(h);
}

int gdc_philox_normals(gdc_handle* h, uint64_t seed, uint32_t c1, uint64_t step, uint32_t c0_begin, int count,
                       double* out) {
  if (!h || !out || count < 0) {
    set_error("handle, output and count >= 0 are required");
    return GDC_EINVAL;
  }
  if (count == 0) return GDC_OK;
  DeviceGuard dg(h->device);
  double* d = nullptr;
  GDC_TRY(dalloc(&d, 4 * (size_t)count));
  int rc = philox_normals_dev(seed, c1, step, c0_begin, count, d, h->stream);
  if (rc == GDC_OK) {
    const hipError_t e1 = hipMemcpyAsync(out, d, 4 * (size_t)count * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    const hipError_t e2 = hipStreamSynchronize(h->stream);
    if (e1 != hipSuccess || e2 != hipSuccess) {
      set_error("copy of the normals failed");
      rc = GDC_EDEVICE;
    }
  }
  (void)hipFree(d);
  return rc;
}

int gdc_philox_normals_noalloc(gdc_handle* h, uint64_t seed, uint32_t c1, uint64_t step, uint32_t c0_begin,
                               int count, double* out) {
  if (!h || !out || count < 0) {
    set_error("handle, output and count >= 0 are required");
    return GDC_EINVAL;
  }
  if (count > NOALLOC_MAX_NORMAL_GROUPS) {
    set_error("gdc_philox_normals_noalloc: count " + std::to_string(count) + " exceeds the staging limit of " +
              std::to_string(NOALLOC_MAX_NORMAL_GROUPS) + " groups of four normals");
    return GDC_EINVAL;
  }
  if (count == 0) return GDC_OK;
  DeviceGuard dg(h->device);
  void* sp = nullptr;
  GDC_TRY(scratch_address(h->device, &sp));
  double* d = static_cast<double*>(sp);
  // every staged value is written by the kernel before it is copied out:
  // nothing to clear
  GDC_TRY(philox_normals_dev(seed, c1, step, c0_begin, count, d, h->stream));
  GDC_HIP(hipMemcpyAsync(out, d, 4 * (size_t)count * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  GDC_HIP(hipStreamSynchronize(h->stream));
  return GDC_OK;
}

}  // extern "C"
