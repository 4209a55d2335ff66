// C-ABI layer of libscfft: argument checking, the workspace, the pass
// schedule of the right-hand side, the device integrator and the readouts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/scfft.h"
#include "bs23.h"
#include "host_model.h"
#include "internal.h"

using namespace scfft;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxDeltaSlots = 256;
constexpr int kIterChunk = 4;  // adaptive iteration: launches between reads of the stop flag
constexpr int kProbeChunk = 4096;
// Per-instance scalars of a batched launch, in each member's workspace (the
// passes read slot [0..3], the batched integrator [4..7], the applied-field
// rates of a plain batched call [8..16], a zero step index [17] and the
// error norm [18]):
enum BPar : int {
  BP_N = 0, BP_RHO, BP_C2, BP_C3,      // n, rho_out, stage coefficients dt/2, 3dt/4
  BP_B1, BP_B2, BP_B3, BP_DT,          // 2dt/9, dt/3, 4dt/9, dt (dimensionless)
  BP_HEDOT = 8,                        // 3 stages x 3 components
  BP_ZERO = 17, BP_ERR = 18,
  kBParDoubles = 32
};

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// FFT lengths: powers of two in [8, 512] and 3 * 2^k in [24, 192].
bool fft_length_supported(int n) {
  auto pow2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
  if (n % 3 == 0) return pow2(n / 3) && n >= 24 && n <= 192;
  return pow2(n) && n >= 8 && n <= 512;
}

}  // namespace

struct scfft_ctx {
  scfft_grid grid;
  scfft_material mat;
  scfft_precision prec;
  hipStream_t stream;
  int device;
  int n[3];
  size_t nodes;
  double L[3];     // dimensionless half widths
  double h[3];     // dimensionless cell sizes
  Units u;
  Drive drive;
  bool has_drive = false;
  scfft_rhs_opts opts;
  double sigma;

  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t off_main, off_warm, off_chi, off_kappa, off_tab, off_part, off_scal, off_delta,
      off_clamp, off_mom, off_adj, off_adjs, off_ode, off_probe, off_bpar, total;
  size_t wsize;  // element size
  bool has_mask = false, has_kappa = false, has_warm = false;
  int64_t n_in = 0, n_out = 0;
  int box_lo[3] = {0, 0, 0}, box_hi[3] = {0, 0, 0};  // index bounding box of Omega (x, y, z)
  int64_t betti[3] = {0, 0, 0};                      // of the mask's voxel union
  std::string err;
  int64_t clamp_seen = 0;
  int iter_guess = 0;  // exterior iterations of the last converged adaptive call
  // where the last adaptive integration stopped, for scfft_ode_opts.resume:
  // its k1 then sits in the K1 slot of the ODE buffers
  Bs23Cont cont;
  // integrator: state whose moment partials the last power-law pass recorded,
  // and whether an observer callback is running (scfft_step_moment)
  const void* mom_state = nullptr;
  const void* obs_state = nullptr;  // state shown to the running observer, else null
  // moment sums (all nodes, Omega) of mom_state, read back with the step's
  // error norm in one transfer; valid while mom_sums_for == mom_state
  double mom_sums[6] = {0, 0, 0, 0, 0, 0};
  const void* mom_sums_for = nullptr;
  // fixed-step integrator: two pinned readback slots (error norm + moment
  // sums, 8 doubles each) and their events, made on first use
  double* rb_pin = nullptr;
  hipEvent_t rb_ev[2] = {nullptr, nullptr};

  // graph-replayed fixed-step integration (scfft_integrate_graph): while a
  // step is captured, passes take their stop flag and applied-field rates
  // from these device locations
  const int* graph_stop = nullptr;
  const double* g_hedot_tab = nullptr;
  const int* g_hedot_step = nullptr;
  int g_hedot_stage = 0;
  double field_hk_inv = 0.0, field_alpha = 0.0;  // e(j, h): 1/h_K (dimensionless), exponent
  double aniso_w[3] = {1.0, 1.0, 1.0};             // anisotropic law weights
  bool has_aniso = false;
  bool graph_busy = false;          // an integration is enqueued; scfft_integrate_wait ends it
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
  // Captured step graphs are kept for the next graph integration with the same
  // workspace, step count and step size; every call that changes what the
  // kernels are launched with (mask, jc map, field law, options, drive,
  // workspace) bumps the epoch and so forces a new capture.
  uint64_t epoch = 1;
  struct {
    const char* gws = nullptr;
    int steps = 0;
    double dt = 0.0;
    uint64_t epoch = 0;
  } graph_key;
  std::vector<double> graph_hedot;  // host copy of the rate table (alive until the wait)
  char* graph_ws = nullptr;
  int graph_steps = 0;
  int graph_accepted = -1;  // steps accepted by the last waited graph integration
  double graph_t0 = 0.0, graph_dt = 0.0;
  void* graph_h = nullptr;

  // optional per-kernel timing with HIP events on the context stream
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;          // pairs: 2i (start), 2i+1 (stop)
  std::vector<int> ev_kind;                 // kind of pending pair i
  size_t ev_used = 0;
  int64_t prof_launches[SCFFT_KERNEL_KINDS] = {};
  double prof_ms[SCFFT_KERNEL_KINDS] = {};
  double prof_bytes[SCFFT_KERNEL_KINDS] = {};  // algorithmic bytes of the timed launches
};

namespace {

scfft_status fail(scfft_ctx* c, scfft_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

// Vector fields are read and written two nodes per access (x = 2i, 2i+1).
bool field_aligned(const scfft_ctx* c, const void* p) {
  return p == nullptr || ((uintptr_t)p) % (2 * c->wsize) == 0;
}

#define CHECK_FIELD(ctx, p)                                                                \
  do {                                                                                     \
    if (!field_aligned(ctx, p))                                                            \
      return fail(ctx, SCFFT_ERR_ARG, "%s is not %zu-byte aligned", #p, 2 * (ctx)->wsize); \
  } while (0)

// The controller continuation belongs to the state the last integration
// ended with; anything that changes the right-hand side or the warm start
// drops it.
void drop_cont(scfft_ctx* c) { c->cont = Bs23Cont{}; }

#define HIPCHK(ctx, call)                                                                  \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, SCFFT_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(e_));          \
  } while (0)

void layout(scfft_ctx* c) {
  const size_t nodes = c->nodes;
  const size_t w = c->wsize;
  const size_t M = (size_t)c->n[0] / 2;
  size_t o = 0;
  c->off_main = o;  o = align_up(o + 3 * (size_t)c->n[2] * c->n[1] * M * 2 * w);
  c->off_warm = o;  o = align_up(o + 3 * nodes * w);
  c->off_chi = o;   o = align_up(o + nodes);
  c->off_kappa = o; o = align_up(o + nodes * w);
  c->off_tab = o;
  for (int a = 0; a < 3; ++a) o = align_up(o + (size_t)c->n[a] * (2 + 3) * w);
  // partials: enough for the X pass (3 per block) and the streaming reductions
  const size_t xb = (size_t)c->n[1] * c->n[2];  // rows: an upper bound of X-pass blocks
  c->off_part = o;  o = align_up(o + std::max<size_t>(3 * xb, 2 * kReduceBlocks) * sizeof(double));
  c->off_scal = o;  o = align_up(o + 16 * sizeof(double));
  c->off_delta = o; o = align_up(o + kMaxDeltaSlots * sizeof(double));
  c->off_clamp = o; o = align_up(o + sizeof(unsigned long long));
  // moment partials of the power-law pass (6 per block) and their sums
  c->off_mom = o;   o = align_up(o + (6 * xb + 8) * sizeof(double));
  // reverse mode: j of the forward call and the running sum of adjoint
  // iterates (one field each), and device accumulators of scalar gradients
  c->off_adj = o;   o = align_up(o + 2 * 3 * nodes * w);
  c->off_adjs = o;  o = align_up(o + 16 * sizeof(double));
  c->off_ode = o;   o = align_up(o + 7 * 3 * nodes * w);  // 6 BS23 fields + a third state
  c->off_probe = o; o = align_up(o + (size_t)kProbeChunk * 6 * sizeof(double));
  // per-instance scalars of a batched launch (scfft_batch): see BPar
  c->off_bpar = o;  o = align_up(o + kBParDoubles * sizeof(double));
  c->total = o;
}

template <typename T>
T* wsp(scfft_ctx* c, size_t off) { return reinterpret_cast<T*>(c->ws + off); }

// Plan over a spectrum at `main` and axis tables at `tab` (per axis: N
// twiddles, then kodd, kk, sm, each N values; axes 256-byte aligned).
template <typename T>
Plan<T> plan_on(const scfft_ctx* c, char* main, char* tab) {
  Plan<T> p;
  p.nx = c->n[0];
  p.ny = c->n[1];
  p.nz = c->n[2];
  p.main = reinterpret_cast<C2<T>*>(main);
  size_t o = 0;
  AxisTab<T>* tabs[3] = {&p.ax, &p.ay, &p.az};
  for (int a = 0; a < 3; ++a) {
    const size_t N = c->n[a];
    tabs[a]->tw = reinterpret_cast<const C2<T>*>(tab + o);
    tabs[a]->kodd = reinterpret_cast<const T*>(tab + o + N * 2 * sizeof(T));
    tabs[a]->kk = reinterpret_cast<const T*>(tab + o + N * 3 * sizeof(T));
    tabs[a]->sm = reinterpret_cast<const T*>(tab + o + N * 4 * sizeof(T));
    o = align_up(o + N * 5 * sizeof(T));
  }
  p.full_ranges();
  p.stop = c->graph_stop;
  p.xalt = c->opts.x_alt;
  p.yalt = c->opts.y_alt;
  p.zalt = c->opts.z_alt;
  return p;
}

template <typename T>
Plan<T> make_plan(scfft_ctx* c) { return plan_on<T>(c, c->ws + c->off_main, c->ws + c->off_tab); }

// Plans restricted to the bounding box of Omega (identical results: skipped
// inputs are exact zeros, skipped outputs are never read).
template <typename T>
struct BoxPlans {
  Plan<T> full;
  Plan<T> z_store;    // Z pass: store only the box planes (output masked to Omega next)
  Plan<T> y_inv;      // Y inverse: box planes, store box rows
  Plan<T> x_box;      // X pass: box rows only
  Plan<T> y_fwd;      // Y forward of a field zero outside the box
  Plan<T> z_load;     // Z pass of a field zero outside the box planes
  Plan<T> x_hin;      // X_HIN with a warm start: inverse only on box rows
  Plan<T> xy_box;     // fused plane pass on box planes only
  Plan<T> xy_hin;     // fused X_HIN: all planes, inverse on box planes
};

template <typename T>
BoxPlans<T> box_plans_for(const int lo[3], const int hi[3], const Plan<T>& p, bool prune) {
  BoxPlans<T> b{p, p, p, p, p, p, p, p, p};
  if (!prune) return b;
  const int y0 = lo[1], y1 = hi[1], z0 = lo[2], z1 = hi[2];
  b.z_store.r.zlo_out = z0;
  b.z_store.r.zhi_out = z1;
  b.y_inv.r.zlo = z0;
  b.y_inv.r.zhi = z1;
  b.y_inv.r.ylo_out = y0;
  b.y_inv.r.yhi_out = y1;
  b.x_box.r.xylo = y0;
  b.x_box.r.xyhi = y1;
  b.x_box.r.xzlo = z0;
  b.x_box.r.xzhi = z1;
  b.y_fwd.r.zlo = z0;
  b.y_fwd.r.zhi = z1;
  b.y_fwd.r.ylo_in = y0;
  b.y_fwd.r.yhi_in = y1;
  b.z_load.r.zlo = z0;
  b.z_load.r.zhi = z1;
  b.x_hin.r.iylo = y0;
  b.x_hin.r.iyhi = y1;
  b.x_hin.r.izlo = z0;
  b.x_hin.r.izhi = z1;
  b.xy_box.r.zlo = z0;
  b.xy_box.r.zhi = z1;
  b.xy_box.r.izlo = z0;
  b.xy_box.r.izhi = z1;
  b.xy_box.r.xylo = y0;  // the mask step transforms only the box rows
  b.xy_box.r.xyhi = y1;
  b.xy_hin.r.izlo = z0;
  b.xy_hin.r.izhi = z1;
  return b;
}

template <typename T>
BoxPlans<T> box_plans(const scfft_ctx* c, const Plan<T>& p, bool prune) {
  return box_plans_for<T>(c->box_lo, c->box_hi, p, prune);
}

// Axis tables in FP64 on the host (Sec. 2: wavenumbers on the box, Gaussian
// smoothing with sigma = half the cell diagonal), converted to T.
template <typename T>
std::vector<char> build_tables(const scfft_ctx* c) {
  std::vector<char> buf(c->off_part - c->off_tab, 0);
  size_t o = 0;
  for (int a = 0; a < 3; ++a) {
    const int N = c->n[a];
    T* tw = reinterpret_cast<T*>(buf.data() + o);
    T* kodd = tw + 2 * N;
    T* kk = tw + 3 * N;
    T* sm = tw + 4 * N;
    for (int i = 0; i < N; ++i) {
      const double ang = -2.0 * M_PI * (double)i / (double)N;
      tw[2 * i] = (T)std::cos(ang);
      tw[2 * i + 1] = (T)std::sin(ang);
      const int m = i < N / 2 ? i : i - N;
      const double k = M_PI * (double)m / c->L[a];
      kodd[i] = (T)(i == N / 2 ? 0.0 : k);
      kk[i] = (T)(k * k);
      sm[i] = (T)std::exp(-0.5 * c->sigma * c->sigma * k * k);
    }
    o = align_up(o + (size_t)N * 5 * sizeof(T));
  }
  return buf;
}

bool ready(scfft_ctx* c, bool need_mask, scfft_status* st) {
  if (c->graph_busy) {
    *st = fail(c, SCFFT_ERR_STATE, "a graph integration is enqueued: call scfft_integrate_wait first");
    return false;
  }
  if (!c->ws) {
    *st = fail(c, SCFFT_ERR_WORKSPACE, "no workspace attached");
    return false;
  }
  if (need_mask && !c->has_mask) {
    *st = fail(c, SCFFT_ERR_GEOMETRY, "no mask: call scfft_voxelize or scfft_set_mask");
    return false;
  }
  return true;
}

// ---------------------------------------------------------------------------
// the right-hand side: pass schedule
// ---------------------------------------------------------------------------
template <typename T>
XArgs<T> base_args(scfft_ctx* c) {
  XArgs<T> a;
  std::memset(&a, 0, sizeof a);
  a.chi = wsp<uint8_t>(c, c->off_chi);
  a.kappa = c->has_kappa ? wsp<T>(c, c->off_kappa) : nullptr;
  a.partials = wsp<double>(c, c->off_part);
  a.clamps = wsp<unsigned long long>(c, c->off_clamp);
  a.hedot_tab = c->g_hedot_tab;
  a.hedot_step = c->g_hedot_step;
  a.hedot_stage = c->g_hedot_stage;
  a.hk_inv = (T)c->field_hk_inv;
  a.kim_alpha = (T)c->field_alpha;
  a.aniso = c->has_aniso ? 1 : 0;
  for (int d = 0; d < 3; ++d) a.aniso_w[d] = (T)c->aniso_w[d];
  a.npow = (T)c->mat.n_power;
  a.rho_out = (T)c->mat.rho_out;
  a.expmax = sizeof(T) == 4 ? (T)80.0 : (T)700.0;
  for (int d = 0; d < 3; ++d) {
    a.pos0[d] = -c->L[d] + 0.5 * c->h[d];
    a.step[d] = c->h[d];
  }
  return a;
}

// ---- per-kernel event timing (scfft_profile) ----
hipError_t prof_harvest(scfft_ctx* c) {
  for (size_t i = 0; i < c->ev_used; ++i) {
    hipError_t e = hipEventSynchronize(c->ev_pool[2 * i + 1]);
    if (e != hipSuccess) return e;
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, c->ev_pool[2 * i], c->ev_pool[2 * i + 1]);
    if (e != hipSuccess) return e;
    c->prof_ms[c->ev_kind[i]] += ms;
    c->prof_launches[c->ev_kind[i]] += 1;
  }
  c->ev_used = 0;
  return hipSuccess;
}

// Event pair for the next launch of `kind` (none when timing is off).
hipError_t prof_slot(scfft_ctx* c, int kind, KTime* t, double bytes) {
  *t = KTime{};
  if (!c->prof) return hipSuccess;
  c->prof_bytes[kind] += bytes;
  if (2 * (c->ev_used + 1) > c->ev_pool.size()) {
    hipError_t e = prof_harvest(c);  // waits for the pending launches
    if (e != hipSuccess) return e;
  }
  c->ev_kind[c->ev_used] = kind;
  t->start = c->ev_pool[2 * c->ev_used];
  t->stop = c->ev_pool[2 * c->ev_used + 1];
  ++c->ev_used;
  return hipSuccess;
}

hipError_t prof_done(scfft_ctx* c, hipError_t launch_err, const KTime& t) {
  if (launch_err != hipSuccess && t.start) --c->ev_used;  // that pair was never recorded
  return launch_err;
}

// Algorithmic bytes of one pass launch: one read of what it must read and one
// write of what it must write, for the launch's ranges.  w = word size; the
// mask-dependent terms use the node counts of Omega and Omega_out.
template <typename T>
double bytes_y(const scfft_ctx* c, const Plan<T>& p) {
  const double cw = 2.0 * sizeof(T), kx = p.nx / 2;
  const double planes = 3.0 * (p.r.zhi - p.r.zlo);
  return p.batch * planes * kx * cw * ((p.r.yhi_in - p.r.ylo_in) + (p.r.yhi_out - p.r.ylo_out));
}
template <typename T>
double bytes_z(const scfft_ctx* c, const Plan<T>& p) {
  const double cw = 2.0 * sizeof(T), col = 3.0 * p.ny * (p.nx / 2);
  return p.batch * col * cw * ((p.r.zhi - p.r.zlo) + (p.r.zhi_out - p.r.zlo_out));
}
template <typename T>
double bytes_x(const scfft_ctx* c, const Plan<T>& p, int op, const XArgs<T>& a) {
  const double w = sizeof(T), cw = 2.0 * w, kx = p.nx / 2;
  const double rows = (double)(p.r.xyhi - p.r.xylo) * (p.r.xzhi - p.r.xzlo);
  const double inv_rows = (double)std::max(0, std::min(p.r.xyhi, p.r.iyhi) - std::max(p.r.xylo, p.r.iylo)) *
                          std::max(0, std::min(p.r.xzhi, p.r.izhi) - std::max(p.r.xzlo, p.r.izlo));
  const double spec = 3.0 * kx * cw;            // one row of the spectrum, 3 components
  const double mask = (double)p.nx;             // one row of the mask
  const double node = 3.0 * w;                  // one node of a real field
  const double nin = (double)c->n_in, nout = (double)c->n_out, all = nin + nout;
  const double frac = rows / ((double)p.ny * p.nz);  // share of the rows in the launch
  switch (op) {
    case X_FWD: return (a.in2 ? 2.0 : 1.0) * rows * p.nx * node + rows * spec;
    case X_LAW: return inv_rows * spec + rows * mask + rows * spec +
                       (a.hk_inv > 0 ? (a.in2 ? 2.0 : 1.0) * nin * frac * node : 0.0) +
                       (a.j_out ? rows * p.nx * node : 0.0);
    case X_HIN: return inv_rows * spec + rows * mask + (a.warm ? nout * frac * node : 0.0) +
                       (a.track ? all : nin) * frac * node + rows * spec;
    case X_MASK: return inv_rows * spec + rows * mask + rows * spec;
    case X_UPDATE: return inv_rows * spec + rows * mask + (a.track ? all + nout : nin) * frac * node +
                          rows * spec;
    case X_UPDATE_LAST: return inv_rows * spec + rows * mask +
                               ((a.track ? all : 0.0) + (a.warm_out ? 2.0 : 1.0) * nout) * frac * node;
    case X_STORE: return inv_rows * spec + rows * p.nx * node;
    case X_MOMENT: return inv_rows * spec + (a.omega_only ? rows * mask : 0.0);
    case X_ADJ_START: return rows * mask + rows * p.nx * node + (a.in2 ? nout * frac * node : 0.0) +
                             rows * p.nx * node + rows * spec;
    case X_ADJ_ACC: return inv_rows * spec + rows * mask + 2.0 * rows * p.nx * node + rows * spec;
    case X_ADJ_LAST: return inv_rows * spec + rows * mask + (a.warm_out ? 2.0 : 1.0) * rows * p.nx * node +
                            rows * spec;
    case X_ADJ_LAW: return inv_rows * spec + rows * mask + nin * frac * node +
                           (a.kappa ? (a.kappa_bar ? 3.0 : 1.0) * nin * frac * w : 0.0) + rows * spec;
  }
  return 0.0;
}
template <typename T>
double bytes_xy(const scfft_ctx* c, const Plan<T>& p, int op, const XArgs<T>& a) {
  // per component plane: spectrum in/out, mask and real-field terms as in X
  const double w = sizeof(T), cw = 2.0 * w, kx = p.nx / 2;
  const double planes = p.r.zhi - p.r.zlo;
  const double inv_planes = std::max(0, std::min(p.r.zhi, p.r.izhi) - std::max(p.r.zlo, p.r.izlo));
  const double spec = 3.0 * p.ny * kx * cw, mask = 3.0 * (double)p.nx * p.ny, node = 3.0 * w;
  const double nin = (double)c->n_in, nout = (double)c->n_out, all = nin + nout;
  const double frac = planes / p.nz;
  switch (op) {
    case XY_FWD: return (a.in2 ? 2.0 : 1.0) * planes * p.ny * p.nx * node + planes * spec;
    case XY_HIN: return inv_planes * spec + planes * mask + (a.warm ? nout * frac * node : 0.0) +
                        (a.track ? all : nin) * frac * node + planes * spec;
    case XY_MASK: return inv_planes * spec + planes * mask * (p.r.xyhi - p.r.xylo) / p.ny + planes * spec;
    case XY_UPDATE: return inv_planes * spec + planes * mask + nin * frac * node + planes * spec;
    case XY_UPDATE_LAST: return inv_planes * spec + planes * mask +
                                (a.warm_out ? 2.0 : 1.0) * nout * frac * node;
    case XY_STORE: return inv_planes * spec + planes * p.ny * p.nx * node;
  }
  return 0.0;
}

template <typename T>
hipError_t run_x(scfft_ctx* c, const Plan<T>& p, int op, const XArgs<T>& a) {
  KTime t;
  const int kind = op < X_ADJ_START ? SCFFT_KERNEL_X_FWD + op : SCFFT_KERNEL_X_ADJ_START + (op - X_ADJ_START);
  hipError_t e = prof_slot(c, kind, &t, c->prof ? p.batch * bytes_x<T>(c, p, op, a) : 0.0);
  if (e != hipSuccess) return e;
  return prof_done(c, launch_xpass<T>(p, op, a, c->stream, t), t);
}

template <typename T>
hipError_t run_y(scfft_ctx* c, const Plan<T>& p, bool inv) {
  KTime t;
  hipError_t e = prof_slot(c, inv ? SCFFT_KERNEL_Y_INV : SCFFT_KERNEL_Y_FWD, &t,
                           c->prof ? bytes_y<T>(c, p) : 0.0);
  if (e != hipSuccess) return e;
  return prof_done(c, launch_ypass<T>(p, inv, c->stream, t), t);
}

template <typename T>
hipError_t run_z(scfft_ctx* c, const Plan<T>& p, int sym, double coef) {
  KTime t;
  hipError_t e = prof_slot(c, sym == Z_CURL ? SCFFT_KERNEL_Z_CURL : SCFFT_KERNEL_Z_PHI, &t,
                           c->prof ? bytes_z<T>(c, p) : 0.0);
  if (e != hipSuccess) return e;
  return prof_done(c, launch_zpass<T>(p, sym, (T)coef, c->stream, t), t);
}

template <typename T>
hipError_t run_xy(scfft_ctx* c, const Plan<T>& p, int op, const XArgs<T>& a) {
  KTime t;
  hipError_t e = prof_slot(c, SCFFT_KERNEL_XY_FWD + op, &t, c->prof ? p.batch * bytes_xy<T>(c, p, op, a) : 0.0);
  if (e != hipSuccess) return e;
  return prof_done(c, launch_xypass<T>(p, op, a, c->stream, t), t);
}

// Y forward, Z (symbol), Y inverse: the middle of one operator application.
template <typename T>
hipError_t spectral_middle(scfft_ctx* c, const Plan<T>& p, int sym, double coef) {
  hipError_t e;
  if ((e = run_y<T>(c, p, false)) != hipSuccess) return e;
  if ((e = run_z<T>(c, p, sym, coef)) != hipSuccess) return e;
  return run_y<T>(c, p, true);
}

// fuse_xy: 0 never, 1 where the fused plane pass measured faster (planes of
// up to 64 x 64 nodes, both precisions; at 128 x 128 the row/column passes
// win: one 133 KB FP64 or 67 KB FP32 plane per block leaves too few waves per
// CU), 2 always (if it fits).
template <typename T>
bool use_xy(const scfft_ctx* c, const Plan<T>& p) {
  if (!xypass_supported<T>(p)) return false;
  return c->opts.fuse_xy >= 2 || (c->opts.fuse_xy == 1 && p.nx <= 64);
}

// The passes of one right-hand side with a fixed iteration count (Sec. 2:
// Eqs. 4, 1, 3, then iteration (5) fixed_iter times), for one context or a
// batch of same-size instances (plan and arguments batched; lo/hi: the box
// that holds Omega of every instance).  With fused xy-plane passes the
// per-component steps (warm start, masks, exterior update) each take one pass
// over the spectrum instead of three; the power law, which needs |j| over the
// three components, keeps the Y inverse / X / Y forward sequence.
template <typename T>
scfft_status rhs_fixed_passes(scfft_ctx* c, const Plan<T>& p, XArgs<T> a, bool warm_start, T* warm,
                              const int lo[3], const int hi[3], const T* h, T* hdot) {
  const double norm = 1.0 / ((double)c->n[0] * c->n[1] * c->n[2]);
  const int phi_sym = c->opts.smooth_phi ? Z_PHI_SMOOTH : Z_PHI;
  const int fixed = c->opts.fixed_iter;
  const BoxPlans<T> b = box_plans_for<T>(lo, hi, p, c->opts.prune_box != 0);
  a.in = h;
  a.out = hdot;
  a.track = 0;
  if (use_xy<T>(c, p)) {
    HIPCHK(c, run_xy<T>(c, p, XY_FWD, a));                     // F(h) in x, y
    HIPCHK(c, run_z<T>(c, p, Z_CURL, norm));                   // j = C_s h (Eq. 4)
    HIPCHK(c, run_y<T>(c, p, true));
    HIPCHK(c, run_x<T>(c, p, X_LAW, a));                       // e (Eq. 1)
    HIPCHK(c, run_y<T>(c, p, false));
    // -C_s e (Eq. 3); with a warm start it is needed on Omega only
    HIPCHK(c, run_z<T>(c, warm_start ? b.z_store : p, Z_CURL, -norm));
    a.warm = warm_start ? warm : nullptr;
    HIPCHK(c, run_xy<T>(c, warm_start ? b.xy_hin : p, XY_HIN, a));  // hdot^0
    for (int it = 0; it < fixed; ++it) {                       // iteration (5)
      HIPCHK(c, run_z<T>(c, b.z_store, Z_CURL, norm));         // jdot^i (needed on Omega)
      HIPCHK(c, run_xy<T>(c, b.xy_box, XY_MASK, a));           // jdot_in^i
      HIPCHK(c, run_z<T>(c, b.z_load, phi_sym, norm));         // Phi[jdot_in^i] (Eq. 7)
      const bool last = it + 1 == fixed;
      a.warm_out = last ? warm : nullptr;
      HIPCHK(c, run_xy<T>(c, p, last ? XY_UPDATE_LAST : XY_UPDATE, a));
    }
    return SCFFT_OK;
  }
  // j = C_s h  (Eq. 4)
  HIPCHK(c, run_x<T>(c, p, X_FWD, a));
  HIPCHK(c, spectral_middle<T>(c, p, Z_CURL, norm));
  // e (Eq. 1; rho_out j outside), then -C_s e (Eq. 3); with a warm start it
  // is needed on Omega only
  HIPCHK(c, run_x<T>(c, p, X_LAW, a));
  HIPCHK(c, run_y<T>(c, p, false));
  HIPCHK(c, run_z<T>(c, warm_start ? b.z_store : p, Z_CURL, -norm));
  HIPCHK(c, run_y<T>(c, warm_start ? b.y_inv : p, true));
  // hdot^0: -curl e on Omega, warm start (or Ohm's law) on Omega_out
  a.warm = warm_start ? warm : nullptr;
  HIPCHK(c, run_x<T>(c, warm_start ? b.x_hin : p, X_HIN, a));
  for (int it = 0; it < fixed; ++it) {  // iteration (5)
    const bool last = it + 1 == fixed;
    // jdot^i = C_s hdot^i (needed on Omega only), jdot_in^i, then Phi[jdot_in^i]
    // (Eq. 7) of a field that vanishes outside the box, update (Eq. 5); the
    // last update also stores the next warm start
    a.warm_out = last ? warm : nullptr;
    HIPCHK(c, run_y<T>(c, p, false));
    HIPCHK(c, run_z<T>(c, b.z_store, Z_CURL, norm));
    HIPCHK(c, run_y<T>(c, b.y_inv, true));
    HIPCHK(c, run_x<T>(c, b.x_box, X_MASK, a));
    HIPCHK(c, run_y<T>(c, b.y_fwd, false));
    HIPCHK(c, run_z<T>(c, b.z_load, phi_sym, norm));
    HIPCHK(c, run_y<T>(c, p, true));
    HIPCHK(c, run_x<T>(c, p, last ? X_UPDATE_LAST : X_UPDATE, a));
  }
  return SCFFT_OK;
}

template <typename T>
// The state is h + in2_coef * in2 (in2 may be null: a Runge-Kutta stage
// argument is formed inside the first pass).  mom: if set, the power-law
// pass also records moment partials of that state (6 per block).
scfft_status rhs_impl(scfft_ctx* c, double t, const T* h, T* hdot, scfft_rhs_stats* stats,
                      const T* in2 = nullptr, double in2_coef = 0.0, double* mom = nullptr,
                      T* j_out = nullptr) {
  const Plan<T> p = make_plan<T>(c);
  const hipStream_t s = c->stream;
  const double norm = 1.0 / ((double)c->n[0] * c->n[1] * c->n[2]);
  const int phi_sym = c->opts.smooth_phi ? Z_PHI_SMOOTH : Z_PHI;
  double he[3], hedot[3];
  c->drive.eval(t, he, hedot);
  const double hedot_abs = std::sqrt(hedot[0] * hedot[0] + hedot[1] * hedot[1] + hedot[2] * hedot[2]);
  const double tol = c->opts.delta_it * std::max(hedot_abs, 1.0);
  const int xb = xpass_blocks<T>(p);

  XArgs<T> a = base_args<T>(c);
  for (int d = 0; d < 3; ++d) a.hedot[d] = (T)hedot[d];
  a.in2 = in2;
  a.in2_coef = (T)in2_coef;
  a.mom_partials = mom;
  a.j_out = j_out;

  const int fixed = c->opts.fixed_iter;
  if (fixed > 0) {
    const scfft_status fs = rhs_fixed_passes<T>(c, p, a, c->has_warm, wsp<T>(c, c->off_warm), c->box_lo,
                                                c->box_hi, h, hdot);
    if (fs < 0) return fs;
    c->has_warm = true;
    scfft_status st = SCFFT_OK;
    if (stats) {
      unsigned long long cl = 0;
      HIPCHK(c, hipMemcpyAsync(&cl, wsp<unsigned long long>(c, c->off_clamp), sizeof cl,
                               hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      const int64_t new_clamps = (int64_t)cl - c->clamp_seen;
      c->clamp_seen = (int64_t)cl;
      stats->iters = fixed;
      stats->converged = 1;
      stats->last_delta = -1.0;
      stats->clamps = new_clamps;
      if (new_clamps > 0) st = SCFFT_WARN_CLAMPED;
    }
    return st;
  }
  const BoxPlans<T> b = box_plans<T>(c, p, c->opts.prune_box != 0);
  const bool warm_start = c->has_warm;

  // j = C_s h  (Eq. 4)
  a.in = h;
  HIPCHK(c, run_x<T>(c, p, X_FWD, a));
  HIPCHK(c, spectral_middle<T>(c, p, Z_CURL, norm));
  // e (Eq. 1; rho_out j outside), then -C_s e (Eq. 3)
  HIPCHK(c, run_x<T>(c, p, X_LAW, a));
  // -C_s e (Eq. 3); with a warm start it is needed on Omega only
  HIPCHK(c, run_y<T>(c, p, false));
  HIPCHK(c, run_z<T>(c, warm_start ? b.z_store : p, Z_CURL, -norm));
  HIPCHK(c, run_y<T>(c, warm_start ? b.y_inv : p, true));
  // hdot^0: -curl e on Omega, warm start (or Ohm's law) on Omega_out; every
  // iterate is kept in hdot (the stopping rule compares consecutive ones)
  a.out = hdot;
  a.warm = c->has_warm ? wsp<T>(c, c->off_warm) : nullptr;
  a.track = 1;
  HIPCHK(c, run_x<T>(c, warm_start ? b.x_hin : p, X_HIN, a));

  // iteration (5) with the stopping rule
  unsigned long long clamps_now = 0;
  int it = 0;
  bool converged = false;
  double last = 0.0;
  // one iteration: jdot^i = C_s hdot^i (needed on Omega only), jdot_in^i, then
  // Phi[jdot_in^i] (Eq. 7) of a field that vanishes outside the box, update (Eq. 5)
  auto iteration = [&](const Plan<T>& pp, const BoxPlans<T>& bb, int op) -> hipError_t {
    hipError_t e;
    if ((e = run_y<T>(c, pp, false)) != hipSuccess) return e;
    if ((e = run_z<T>(c, bb.z_store, Z_CURL, norm)) != hipSuccess) return e;
    if ((e = run_y<T>(c, bb.y_inv, true)) != hipSuccess) return e;
    if ((e = run_x<T>(c, bb.x_box, X_MASK, a)) != hipSuccess) return e;
    if ((e = run_y<T>(c, bb.y_fwd, false)) != hipSuccess) return e;
    if ((e = run_z<T>(c, bb.z_load, phi_sym, norm)) != hipSuccess) return e;
    if ((e = run_y<T>(c, pp, true)) != hipSuccess) return e;
    return run_x<T>(c, pp, op, a);
  };
  {
    // Stopping rule on the device: after each update a one-block kernel sums
    // |delta| and sets a stop flag that makes every later pass of the loop
    // return at once.  The host first launches as many iterations as the
    // previous call needed (the warm start makes consecutive calls alike),
    // the last of them in the form that stores hdot and the next warm start
    // without a forward transform, and reads the flag once; only if that
    // was too few does it rebuild the spectrum and go on kIterChunk
    // iterations at a time.
    IterState* ist = wsp<IterState>(c, c->off_delta);
    HIPCHK(c, launch_iter_reset(ist, s));
    Plan<T> pl = p;
    pl.stop = &ist->stop;
    const BoxPlans<T> bl = box_plans<T>(c, pl, c->opts.prune_box != 0);
    const int max_it = std::max(1, c->opts.max_iter);
    const int guess = std::min(max_it, std::max({1, c->opts.min_iter, c->iter_guess > 0 ? c->iter_guess : kIterChunk}));
    IterState hst{0, 0, 0.0};
    auto read_state = [&]() -> hipError_t {
      hipError_t e;
      if ((e = hipMemcpyAsync(&hst, ist, sizeof hst, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
      if ((e = hipMemcpyAsync(&clamps_now, wsp<unsigned long long>(c, c->off_clamp), sizeof clamps_now,
                              hipMemcpyDeviceToHost, s)) != hipSuccess)
        return e;
      return hipStreamSynchronize(s);
    };
    auto copy_warm = [&]() {  // warm start of the next call, read on Omega_out only
      return hipMemcpyAsync(wsp<T>(c, c->off_warm), hdot, 3 * c->nodes * sizeof(T), hipMemcpyDeviceToDevice, s);
    };
    for (int k = 0; k < guess; ++k) {
      const bool lastk = k + 1 == guess;
      a.warm_out = lastk ? wsp<T>(c, c->off_warm) : nullptr;
      HIPCHK(c, iteration(pl, bl, lastk ? X_UPDATE_LAST : X_UPDATE));
      HIPCHK(c, launch_iter_decide(a.partials, xb, (double)c->n_out, tol, c->opts.min_iter, ist, s));
    }
    a.warm_out = nullptr;
    int launched = guess;
    HIPCHK(c, read_state());
    if (hst.stop) {
      if (hst.iters < guess) HIPCHK(c, copy_warm());  // the storing update did not run
    } else if (launched < max_it) {
      // the spectrum of hdot for the next iteration (the storing update made none)
      a.in = hdot;
      a.in2 = nullptr;
      HIPCHK(c, run_x<T>(c, p, X_FWD, a));
      while (launched < max_it) {
        const int chunk = std::min(kIterChunk, max_it - launched);
        for (int k = 0; k < chunk; ++k) {
          HIPCHK(c, iteration(pl, bl, X_UPDATE));
          HIPCHK(c, launch_iter_decide(a.partials, xb, (double)c->n_out, tol, c->opts.min_iter, ist, s));
        }
        launched += chunk;
        HIPCHK(c, read_state());
        if (hst.stop || launched >= max_it) {
          HIPCHK(c, copy_warm());
          break;
        }
      }
    }
    if (hst.stop) c->iter_guess = hst.iters;
    it = hst.iters;
    last = hst.last;
    converged = hst.stop != 0;
  }
  c->has_warm = true;

  scfft_status st = converged ? SCFFT_OK : SCFFT_WARN_NOT_CONVERGED;
  // the adaptive loop read the clamp counter with its last flag
  const int64_t new_clamps = (int64_t)clamps_now - c->clamp_seen;
  c->clamp_seen = (int64_t)clamps_now;
  if (stats) {
    stats->iters = it;
    stats->converged = converged ? 1 : 0;
    stats->last_delta = last;
    stats->clamps = new_clamps;
  }
  if (st == SCFFT_OK && new_clamps > 0) st = SCFFT_WARN_CLAMPED;
  return st;
}

// Reverse mode of one right-hand-side call with a fixed iteration count K,
// the transpose of (h, w) -> (hdot, w' = (1-chi) hdot), w the warm start.
// The curl and Phi have Hermitian symbols (symmetric operators), the masks
// are diagonal and the Jacobian of Eq. 1 is symmetric, so the passes of the
// forward schedule run in reverse order:
//   l^K = lam + (1-chi) mu;  l^i = C chi Phi (1-chi) l^{i+1};  c = sum_{i>=1} l^i
//   gbar = chi c + (chi or 1) l^0;  wbar = (1-chi) l^0;  hedot_bar = sum (1-chi) c
//   ebar = -C gbar;  jbar = (de/dj)^T ebar;  hbar = C jbar
// The state is h + in2_coef in2 (a stage argument).  Scalars go to device
// accumulators: sc[0] += nbar, sc[1..3] += rate_scale * hedot_bar;
// kappa_bar (scalar field) is accumulated when non-null.
template <typename T>
// j_known: j = C_s h of the forward call if the caller kept it (else recomputed).
scfft_status rhs_vjp_impl(scfft_ctx* c, const T* h, const T* in2, double in2_coef, bool warm_used,
                          const T* lam, const T* mu, T* hbar, T* wbar, T* kbar, double* sc,
                          double rate_scale, const T* j_known = nullptr) {
  const int K = c->opts.fixed_iter;
  if (K <= 0) return fail(c, SCFFT_ERR_ARG, "reverse mode needs a fixed iteration count (fixed_iter > 0)");
  if (c->field_hk_inv > 0.0)
    return fail(c, SCFFT_ERR_ARG, "reverse mode of the field-dependent law is not implemented");
  if (c->has_aniso)
    return fail(c, SCFFT_ERR_ARG, "reverse mode of the anisotropic law is not implemented");
  const Plan<T> p = make_plan<T>(c);
  const double norm = 1.0 / ((double)c->n[0] * c->n[1] * c->n[2]);
  const int phi_sym = c->opts.smooth_phi ? Z_PHI_SMOOTH : Z_PHI;
  const int xb = xpass_blocks<T>(p);
  T* jbuf = wsp<T>(c, c->off_adj);
  T* acc = jbuf + 3 * c->nodes;
  XArgs<T> a = base_args<T>(c);
  const T* jv = j_known;
  if (!jv) {
    // j = C h at the forward call's state (Eq. 4), taken from the power-law
    // pass as in the forward call (bitwise the same j; its law output and
    // clamp count are discarded)
    a.in = h;
    a.in2 = in2;
    a.in2_coef = (T)in2_coef;
    if (use_xy<T>(c, p)) {  // the forward call's fused schedule (fixed count)
      HIPCHK(c, run_xy<T>(c, p, XY_FWD, a));
      HIPCHK(c, run_z<T>(c, p, Z_CURL, norm));
      HIPCHK(c, run_y<T>(c, p, true));
    } else {
      HIPCHK(c, run_x<T>(c, p, X_FWD, a));
      HIPCHK(c, spectral_middle<T>(c, p, Z_CURL, norm));
    }
    XArgs<T> al = a;
    al.j_out = jbuf;
    al.clamps = reinterpret_cast<unsigned long long*>(wsp<double>(c, c->off_adjs) + 8);
    HIPCHK(c, run_x<T>(c, p, X_LAW, al));
    a.in2 = nullptr;
    jv = jbuf;
  }
  // the exterior iteration (Eq. 5) transposed, last iterate first
  a.in = lam;
  a.in2 = mu;
  a.out = acc;
  HIPCHK(c, run_x<T>(c, p, X_ADJ_START, a));
  a.in2 = nullptr;
  for (int i = K - 1; i >= 0; --i) {
    HIPCHK(c, spectral_middle<T>(c, p, phi_sym, norm));      // Phi (Eq. 7)
    HIPCHK(c, run_x<T>(c, p, X_MASK, a));                     // chi
    HIPCHK(c, spectral_middle<T>(c, p, Z_CURL, norm));        // C
    if (i > 0) {
      HIPCHK(c, run_x<T>(c, p, X_ADJ_ACC, a));
    } else {
      a.warm_out = wbar;
      a.warm_used = warm_used ? 1 : 0;
      HIPCHK(c, run_x<T>(c, p, X_ADJ_LAST, a));
      HIPCHK(c, launch_accum_partials(a.partials, xb, 3, 3, rate_scale, sc + 1, c->stream));
      a.warm_out = nullptr;
    }
  }
  // ebar = -C gbar (Eq. 3); jbar = (de/dj)^T ebar (Eq. 1); hbar = C jbar (Eq. 4)
  HIPCHK(c, spectral_middle<T>(c, p, Z_CURL, -norm));
  a.in = jv;
  a.kappa_bar = kbar;
  HIPCHK(c, run_x<T>(c, p, X_ADJ_LAW, a));
  HIPCHK(c, launch_accum_partials(a.partials, xb, 1, 1, 1.0, sc, c->stream));
  a.kappa_bar = nullptr;
  HIPCHK(c, spectral_middle<T>(c, p, Z_CURL, norm));
  a.out = hbar;
  HIPCHK(c, run_x<T>(c, p, X_STORE, a));
  return SCFFT_OK;
}

// One operator application v -> out: forward transform, the symbol in the Z
// pass, inverse transform (the X/XY passes read in and write out only).
template <typename T>
scfft_status apply_on(scfft_ctx* c, const Plan<T>& p, const XArgs<T>& a, int sym, double sign) {
  const double norm = 1.0 / ((double)c->n[0] * c->n[1] * c->n[2]);
  if (use_xy<T>(c, p)) {
    HIPCHK(c, run_xy<T>(c, p, XY_FWD, a));
    HIPCHK(c, run_z<T>(c, p, sym, sign * norm));
    HIPCHK(c, run_xy<T>(c, p, XY_STORE, a));
    return SCFFT_OK;
  }
  HIPCHK(c, run_x<T>(c, p, X_FWD, a));
  HIPCHK(c, spectral_middle<T>(c, p, sym, sign * norm));
  HIPCHK(c, run_x<T>(c, p, X_STORE, a));
  return SCFFT_OK;
}

template <typename T>
scfft_status apply_operator(scfft_ctx* c, const T* v, T* out, int sym, double sign) {
  XArgs<T> a = base_args<T>(c);
  a.in = v;
  a.out = out;
  return apply_on<T>(c, make_plan<T>(c), a, sym, sign);
}

// ---------------------------------------------------------------------------
// allocation-free curl (scfft_curl_noalloc)
// ---------------------------------------------------------------------------
// For callers that cannot allocate device memory, the half spectrum and the
// axis tables of one curl live in this file-scope device array instead of the
// context's workspace: one copy per GPU, held until the process ends, shared
// by every call on that GPU.  In host code the array's name is not a device
// address: host code uses the address hipGetSymbolAddress returns for the
// current device (scratch_on), looked up once per device.
constexpr size_t kScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_on(int dev, char** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// bytes of the scratch array one curl needs: half spectrum, then the tables
size_t noalloc_spec_bytes(const scfft_ctx* c) {
  return align_up(3 * (size_t)c->n[2] * c->n[1] * (c->n[0] / 2) * 2 * c->wsize);
}
size_t noalloc_bytes(const scfft_ctx* c) {
  size_t o = noalloc_spec_bytes(c);
  for (int a = 0; a < 3; ++a) o = align_up(o + (size_t)c->n[a] * 5 * c->wsize);
  return o;
}

template <typename T>
scfft_status curl_noalloc_impl(scfft_ctx* c, char* base, const T* v, T* out) {
  char* tab = base + noalloc_spec_bytes(c);
  size_t o = 0;
  for (int a = 0; a < 3; ++a) {  // every call writes the tables it reads
    const size_t N = c->n[a];
    HIPCHK(c, launch_axis_table<T>(reinterpret_cast<C2<T>*>(tab + o), reinterpret_cast<T*>(tab + o + N * 2 * sizeof(T)),
                                   reinterpret_cast<T*>(tab + o + N * 3 * sizeof(T)),
                                   reinterpret_cast<T*>(tab + o + N * 4 * sizeof(T)), (int)N, c->L[a], c->sigma,
                                   c->stream));
    o = align_up(o + N * 5 * sizeof(T));
  }
  XArgs<T> a;
  std::memset(&a, 0, sizeof a);  // the forward and store passes read in and write out only
  a.in = v;
  a.out = out;
  return apply_on<T>(c, plan_on<T>(c, base, tab), a, Z_CURL, 1.0);
}

template <typename T>
scfft_status moment_impl(scfft_ctx* c, const T* h, int omega_only, double m[3]) {
  const Plan<T> p = make_plan<T>(c);
  const double norm = 1.0 / ((double)c->n[0] * c->n[1] * c->n[2]);
  XArgs<T> a = base_args<T>(c);
  a.in = h;
  a.omega_only = omega_only ? 1 : 0;
  HIPCHK(c, run_x<T>(c, p, X_FWD, a));
  HIPCHK(c, spectral_middle<T>(c, p, Z_CURL, norm));
  HIPCHK(c, run_x<T>(c, p, X_MOMENT, a));
  double* out = wsp<double>(c, c->off_scal);
  HIPCHK(c, launch_sum_partials(a.partials, xpass_blocks<T>(p), 3, 3, out, c->stream));
  double r[3];
  HIPCHK(c, hipMemcpyAsync(r, out, sizeof r, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const double dv = c->h[0] * c->h[1] * c->h[2];
  const double scale = c->u.jc * std::pow(c->u.l, 4.0);  // m' -> A m^2
  for (int d = 0; d < 3; ++d) m[d] = 0.5 * r[d] * dv * scale;
  return SCFFT_OK;
}

// ---------------------------------------------------------------------------
// device integrator ops
// ---------------------------------------------------------------------------
template <typename T>
struct DeviceOps {
  scfft_ctx* c;
  T* buf[6];
  scfft_observer obs;
  void* user;
  scfft_ode_stats* st;
  scfft_status last_warn = SCFFT_OK;

  // dst = f(t, y + coef k); a state (k = B_NONE) also records its moment
  // partials when an observer may ask for them
  int eval(double t, Buf y, Buf k, double coef, Buf dst) {
    scfft_rhs_stats rs;
    const bool state = k == B_NONE;
    double* mom = state && obs ? wsp<double>(c, c->off_mom) : nullptr;
    scfft_status s = rhs_impl<T>(c, t, buf[y], buf[dst], c->opts.fixed_iter > 0 ? nullptr : &rs,
                                 state ? nullptr : buf[k], state ? 0.0 : coef, mom);
    if (s < 0) return s;
    if (mom) {
      c->mom_state = buf[y];
      c->mom_sums_for = nullptr;  // the sums read so far belong to another state
    }
    if (c->opts.fixed_iter > 0) {
      st->iters_total += c->opts.fixed_iter;
    } else {
      st->iters_total += rs.iters;
      if (!rs.converged) st->not_converged += 1;
      st->clamps += rs.clamps;
    }
    if (s > 0) last_warn = s;
    return 0;
  }
  int rhs(double t, Buf src, Buf dst) { return eval(t, src, B_NONE, 0.0, dst); }
  int rhs_at(double t, Buf y, Buf k, double coef, Buf dst) { return eval(t, y, k, coef, dst); }
  int combo(Buf out, Buf y, Buf a, double ca, Buf b, double cb, Buf cc_, double cc) {
    hipError_t e = launch_combo<T>(buf[out], buf[y], a >= 0 ? buf[a] : nullptr, ca,
                                   b >= 0 ? buf[b] : nullptr, cb, cc_ >= 0 ? buf[cc_] : nullptr, cc,
                                   3 * c->nodes, c->stream);
    return e == hipSuccess ? 0 : fail(c, SCFFT_ERR_DEVICE, "combo: %s", hipGetErrorString(e));
  }
  // The error norm of the step; where the new state y1 recorded moment
  // partials (an observer is set), their sums come back in the same
  // transfer, so the observer's scfft_step_moment costs no second wait.
  int errnorm(Buf y, Buf y1, double dt, double thr, double* err) {
    double* part = wsp<double>(c, c->off_part);
    double* out = wsp<double>(c, c->off_scal);
    const bool with_mom = obs && c->mom_state == buf[y1];
    hipError_t e = launch_errnorm<T>(buf[y], buf[y1], buf[B_K1], buf[B_K2], buf[B_K3], buf[B_K4],
                                     dt, thr, 3 * c->nodes, part, kReduceBlocks, c->stream);
    if (e == hipSuccess) e = launch_max_partials(part, kReduceBlocks, out, c->stream);
    if (e == hipSuccess && with_mom)
      e = launch_sum_partials(wsp<double>(c, c->off_mom), xpass_blocks<T>(make_plan<T>(c)), 6, 6,
                              out + 1, c->stream);
    double r[7];
    const size_t nb = (with_mom ? 7 : 1) * sizeof(double);
    if (e == hipSuccess) e = hipMemcpyAsync(r, out, nb, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(c, SCFFT_ERR_DEVICE, "errnorm: %s", hipGetErrorString(e));
    *err = r[0];
    if (with_mom) {
      for (int k = 0; k < 6; ++k) c->mom_sums[k] = r[1 + k];
      c->mom_sums_for = buf[y1];
    }
    return 0;
  }
  // The same reduction as errnorm, read back into pinned slot `slot`
  // behind an event instead of waited for: the host can enqueue the next
  // step first.  errnorm_wait then waits for that event only.
  const void* pend_mom[2] = {nullptr, nullptr};
  int errnorm_enqueue(Buf y, Buf y1, double dt, double thr, int slot) {
    double* part = wsp<double>(c, c->off_part);
    double* out = wsp<double>(c, c->off_scal);
    const bool with_mom = obs && c->mom_state == buf[y1];
    hipError_t e = launch_errnorm<T>(buf[y], buf[y1], buf[B_K1], buf[B_K2], buf[B_K3], buf[B_K4],
                                     dt, thr, 3 * c->nodes, part, kReduceBlocks, c->stream);
    if (e == hipSuccess) e = launch_max_partials(part, kReduceBlocks, out, c->stream);
    if (e == hipSuccess && with_mom)
      e = launch_sum_partials(wsp<double>(c, c->off_mom), xpass_blocks<T>(make_plan<T>(c)), 6, 6,
                              out + 1, c->stream);
    const size_t nb = (with_mom ? 7 : 1) * sizeof(double);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->rb_pin + 8 * slot, out, nb, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->rb_ev[slot], c->stream);
    if (e != hipSuccess) return fail(c, SCFFT_ERR_DEVICE, "errnorm: %s", hipGetErrorString(e));
    pend_mom[slot] = with_mom ? buf[y1] : nullptr;
    return 0;
  }
  int errnorm_wait(int slot, double* err) {
    const hipError_t e = hipEventSynchronize(c->rb_ev[slot]);
    if (e != hipSuccess) return fail(c, SCFFT_ERR_DEVICE, "errnorm: %s", hipGetErrorString(e));
    const double* r = c->rb_pin + 8 * slot;
    *err = r[0];
    if (pend_mom[slot]) {
      for (int k = 0; k < 6; ++k) c->mom_sums[k] = r[1 + k];
      c->mom_sums_for = pend_mom[slot];
    }
    return 0;
  }
  int rate(double thr, double* r) {
    double* part = wsp<double>(c, c->off_part);
    double* out = wsp<double>(c, c->off_scal);
    hipError_t e = launch_ratio_max<T>(buf[B_K1], buf[B_Y], thr, 3 * c->nodes, part,
                                       kReduceBlocks, c->stream);
    if (e == hipSuccess) e = launch_max_partials(part, kReduceBlocks, out, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(r, out, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? 0 : fail(c, SCFFT_ERR_DEVICE, "rate: %s", hipGetErrorString(e));
  }
  int accept() {  // the state lives in the workspace: swap, no copy
    std::swap(buf[B_Y], buf[B_Y1]);
    std::swap(buf[B_K1], buf[B_K4]);
    return 0;
  }
  int observe(double t, int* stop) {
    *stop = 0;
    if (obs) {
      c->obs_state = buf[B_Y];
      *stop = obs(user, t * c->u.t0, buf[B_Y]);
      c->obs_state = nullptr;
    }
    return 0;
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// host test integrator ops
// ---------------------------------------------------------------------------
namespace {

struct HostOps {
  int64_t n;
  std::vector<double> b[6];
  double* y;
  scfft_host_rhs f;
  void* user;
  double* bp(Buf k) { return k == B_Y ? y : b[k].data(); }
  int rhs(double t, Buf src, Buf dst) {
    return f(user, t, bp(src), bp(dst)) == 0 ? 0 : SCFFT_ERR_ARG;
  }
  int rhs_at(double t, Buf yy, Buf k, double coef, Buf dst) {  // stage argument in Y1
    int r = combo(B_Y1, yy, k, coef, B_NONE, 0.0, B_NONE, 0.0);
    return r < 0 ? r : rhs(t, B_Y1, dst);
  }
  int combo(Buf out, Buf yy, Buf a, double ca, Buf bb, double cb, Buf cc_, double cc) {
    double *o = bp(out), *py = bp(yy);
    double* pa = a >= 0 ? bp(a) : nullptr;
    double* pb = bb >= 0 ? bp(bb) : nullptr;
    double* pc = cc_ >= 0 ? bp(cc_) : nullptr;
    for (int64_t i = 0; i < n; ++i) {
      double v = py[i];
      if (pa) v += ca * pa[i];
      if (pb) v += cb * pb[i];
      if (pc) v += cc * pc[i];
      o[i] = v;
    }
    return 0;
  }
  int errnorm(Buf yy, Buf y1, double dt, double thr, double* err) {
    const double e1 = -5.0 / 72.0, e2 = 1.0 / 12.0, e3 = 1.0 / 9.0, e4 = -1.0 / 8.0;
    double m = 0.0;
    double *k1 = bp(B_K1), *k2 = bp(B_K2), *k3 = bp(B_K3), *k4 = bp(B_K4), *p = bp(yy), *q = bp(y1);
    for (int64_t i = 0; i < n; ++i) {
      const double E = dt * (e1 * k1[i] + e2 * k2[i] + e3 * k3[i] + e4 * k4[i]);
      double r = std::fabs(E) / std::max(std::max(std::fabs(p[i]), std::fabs(q[i])), thr);
      if (!std::isfinite(r)) r = INFINITY;
      m = std::max(m, r);
    }
    *err = m;
    return 0;
  }
  int rate(double thr, double* r) {
    double m = 0.0;
    for (int64_t i = 0; i < n; ++i) m = std::max(m, std::fabs(b[B_K1][i]) / std::max(std::fabs(y[i]), thr));
    *r = m;
    return 0;
  }
  int accept() {
    std::copy(b[B_Y1].begin(), b[B_Y1].end(), y);
    std::swap(b[B_K1], b[B_K4]);
    return 0;
  }
  int observe(double, int* stop) {
    *stop = 0;
    return 0;
  }
};

bool valid_ode_opts(const scfft_ode_opts* o) {
  return o && o->rtol > 0.0 && o->atol > 0.0 && o->dt0_s >= 0.0 && o->dt_max_s >= 0.0 &&
         o->fixed_steps >= 0 && o->n_bp >= 0 && (o->n_bp == 0 || o->breakpoints_s) &&
         o->max_steps >= 0 && (o->resume == 0 || o->resume == 1);
}

// Fixed-step BS23 (the steps of bs23_run's fixed mode) with the next step
// enqueued before the host waits for the current step's error norm and
// moment sums, so the GPU does not idle while the host reads them and runs
// the observer.  A third state buffer keeps the last accepted state intact
// until the step after it has been checked: on a non-finite error norm the
// state is the last accepted one, as in the sequential loop.  An observer
// that stops the run does so after the next step was already computed (its
// result is dropped; the warm start is that of its evaluations).
template <typename T>
scfft_status fixed_steps_pipelined(scfft_ctx* c, DeviceOps<T>& ops, T* third, double t0, double t1,
                                   int nsteps, double rtol, double atol, scfft_ode_stats& st) {
  const double thr = atol / rtol;
  const double dt = (t1 - t0) / nsteps;
  auto t_of = [&](int s) { return s < nsteps ? t0 + s * dt : t1; };
  auto enqueue = [&](int s) -> int {  // step s from buf[B_Y], buf[B_K1] into buf[B_Y1], buf[B_K4]
    const double t = t_of(s), h = t_of(s + 1) - t;
    int r;
    if ((r = ops.rhs_at(t + 0.5 * h, B_Y, B_K1, 0.5 * h, B_K2)) < 0) return r;
    if ((r = ops.rhs_at(t + 0.75 * h, B_Y, B_K2, 0.75 * h, B_K3)) < 0) return r;
    if ((r = ops.combo(B_Y1, B_Y, B_K1, h * (2.0 / 9.0), B_K2, h * (1.0 / 3.0), B_K3,
                       h * (4.0 / 9.0))) < 0)
      return r;
    if ((r = ops.rhs(t + h, B_Y1, B_K4)) < 0) return r;
    st.rhs_calls += 3;
    return ops.errnorm_enqueue(B_Y, B_Y1, h, thr, s & 1);
  };
  int rc;
  if ((rc = ops.rhs(t0, B_Y, B_K1)) < 0) return (scfft_status)rc;
  st.rhs_calls += 1;
  if ((rc = enqueue(0)) < 0) return (scfft_status)rc;
  for (int s = 0; s < nsteps; ++s) {
    // buffers of step s: state y_s in B_Y, y_{s+1} in B_Y1, f(y_s) in B_K1,
    // f(y_{s+1}) in B_K4.  Step s + 1 reads y_{s+1}, f(y_{s+1}) and writes
    // the free state buffer and f(y_s)'s buffer (read by step s only).
    T* prev = ops.buf[B_Y];
    ops.buf[B_Y] = ops.buf[B_Y1];
    ops.buf[B_Y1] = third;
    third = prev;
    std::swap(ops.buf[B_K1], ops.buf[B_K4]);
    if (s + 1 < nsteps && (rc = enqueue(s + 1)) < 0) return (scfft_status)rc;
    double err = 0.0;
    if ((rc = ops.errnorm_wait(s & 1, &err)) < 0) return (scfft_status)rc;
    if (!std::isfinite(err)) {
      ops.buf[B_Y] = prev;  // the last accepted state
      return SCFFT_ERR_NAN;
    }
    st.dt_last_s = t_of(s + 1) - t_of(s);
    st.err_last = err;
    st.t_s = t_of(s + 1);
    st.accepted += 1;
    int stop = 0;
    if ((rc = ops.observe(t_of(s + 1), &stop)) < 0) return (scfft_status)rc;
    if (stop) break;
  }
  return SCFFT_OK;
}

template <typename T>
scfft_status integrate_impl(scfft_ctx* c, double t0, double t1, T* h, const scfft_ode_opts* o,
                            scfft_observer obs, void* user, scfft_ode_stats* st) {
  // the state is integrated in a workspace buffer (accepting a step swaps
  // buffers) and copied back to h at the end, also after a failure
  DeviceOps<T> ops;
  ops.c = c;
  const size_t fb = 3 * c->nodes * sizeof(T);
  for (int k = 0; k < 6; ++k) ops.buf[k] = wsp<T>(c, c->off_ode + (size_t)k * fb);
  ops.obs = obs;
  ops.user = user;
  ops.st = st;
  c->mom_state = nullptr;
  c->mom_sums_for = nullptr;
  HIPCHK(c, hipMemcpyAsync(ops.buf[B_Y], h, fb, hipMemcpyDeviceToDevice, c->stream));
  scfft_ode_opts od = *o;  // convert times to t' = t / t0
  od.dt0_s = o->dt0_s / c->u.t0;
  od.dt_max_s = o->dt_max_s / c->u.t0;
  std::vector<double> stops = c->drive.kinks();
  for (int i = 0; i < o->n_bp; ++i) stops.push_back(o->breakpoints_s[i] / c->u.t0);
  scfft_status s;
  // resume the adaptive controller where the last adaptive integration (or
  // a restored state blob) stopped; its k1 sits in the K1 slot
  Bs23Cont cont = c->cont;
  const double t0d = t0 / c->u.t0;
  cont.use = o->resume && o->fixed_steps <= 0 && cont.valid &&
             std::fabs(cont.t - t0d) <= 1e-12 * std::max(std::fabs(t0d), 1.0);
  drop_cont(c);
  if (o->fixed_steps > 0 && t1 > t0) {
    if (!c->rb_pin) {
      HIPCHK(c, hipHostMalloc((void**)&c->rb_pin, 16 * sizeof(double), hipHostMallocDefault));
      for (auto& e : c->rb_ev) HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    st->t_s = t0 / c->u.t0;
    s = fixed_steps_pipelined<T>(c, ops, wsp<T>(c, c->off_ode + 6 * fb), t0 / c->u.t0, t1 / c->u.t0,
                                 o->fixed_steps, od.rtol, od.atol, *st);
  } else {
    // a resumed run starts at the stored time itself, not at t0_s / t0
    // (which may differ from it in the last bit)
    s = bs23_run(ops, cont.use ? cont.t : t0d, t1 / c->u.t0, od, stops, *st, &cont);
    if (s >= 0 && cont.valid) {
      // keep k1 in the K1 slot, where the next resumed run expects it
      T* slot = wsp<T>(c, c->off_ode + (size_t)B_K1 * fb);
      if (cont.has_k1 && ops.buf[B_K1] != slot)
        HIPCHK(c, hipMemcpyAsync(slot, ops.buf[B_K1], fb, hipMemcpyDeviceToDevice, c->stream));
      cont.use = false;
      c->cont = cont;
    }
  }
  c->mom_state = nullptr;
  c->obs_state = nullptr;
  c->mom_sums_for = nullptr;
  HIPCHK(c, hipMemcpyAsync(h, ops.buf[B_Y], fb, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  st->t_s *= c->u.t0;
  st->dt_last_s *= c->u.t0;
  if (s == SCFFT_OK && st->not_converged > 0) s = SCFFT_WARN_NOT_CONVERGED;
  return s;
}

// ---------------------------------------------------------------------------
// reverse mode of fixed-step BS23
// ---------------------------------------------------------------------------
// Caller workspace: nseg checkpoints (state, k1, warm start at a segment's
// first step), the tape of one segment (per step: state, k1, k2 and the
// current density j = C_s u of the three stage states u2, u3, u4; and the
// state after it), and 10 fields for the forward pass and the cotangents.
struct AdjLayout {
  size_t F = 0;
  int nseg = 0, every = 0;
  size_t off_tape = 0, off_vec = 0, total = 0;
};

AdjLayout adj_layout(const scfft_ctx* c, int steps, int every) {
  AdjLayout L;
  L.F = align_up(3 * (size_t)c->nodes * c->wsize);
  L.every = every;
  L.nseg = (steps + every - 1) / every;
  L.off_tape = (size_t)L.nseg * 3 * L.F;
  L.off_vec = L.off_tape + (size_t)(6 * every + 1) * L.F;
  L.total = L.off_vec + 10 * L.F;
  return L;
}

template <typename T>
struct AdjRun {
  scfft_ctx* c;
  char* ws;
  AdjLayout L;
  T* f(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  T* cp(int seg, int k) const { return f(((size_t)seg * 3 + k) * L.F); }  // k: 0 y, 1 k1, 2 warm
  // k: 0 y, 1 k1, 2 k2, 3 j(u2), 4 j(u3), 5 j(u4)
  T* tape(int m, int k) const { return f(L.off_tape + ((size_t)m * 6 + k) * L.F); }
  T* yend() const { return f(L.off_tape + (size_t)(6 * L.every) * L.F); }
  T* vec(int i) const { return f(L.off_vec + (size_t)i * L.F); }
  size_t fb() const { return 3 * c->nodes * sizeof(T); }

  scfft_status rhs(double t, const T* y, const T* k, double coef, T* out, T* j_out = nullptr) {
    return rhs_impl<T>(c, t, y, out, nullptr, k, coef, nullptr, j_out);
  }
  scfft_status combo(T* out, const T* y, const T* a, double ca, const T* b, double cb, const T* d,
                     double cd) {
    HIPCHK(c, launch_combo<T>(out, y, a, ca, b, cb, d, cd, 3 * c->nodes, c->stream));
    return SCFFT_OK;
  }
  scfft_status copy(T* dst, const T* src) {
    HIPCHK(c, hipMemcpyAsync(dst, src, fb(), hipMemcpyDeviceToDevice, c->stream));
    return SCFFT_OK;
  }
};

#define ADJCHK(call)                  \
  do {                                \
    scfft_status s_ = (call);         \
    if (s_ < 0) return s_;            \
  } while (0)

template <typename T>
scfft_status integrate_adjoint_impl(scfft_ctx* c, double t0, double t1, int steps, int every,
                                    char* ws, T* hT, const T* h0, const T* hT_bar, T* h0_bar, T* kbar,
                                    double* n_bar, double p_bar[3]) {
  AdjRun<T> R{c, ws, adj_layout(c, steps, every)};
  const double dt = (t1 - t0) / steps;
  auto t_of = [&](int s) { return s == 0 ? t0 : (s < steps ? t0 + s * dt : t1); };
  double pv[3];
  for (int d = 0; d < 3; ++d) pv[d] = c->drive.dir[d] * c->drive.amp;
  const double pp = pv[0] * pv[0] + pv[1] * pv[1] + pv[2] * pv[2];
  auto rate = [&](double t) {  // f'(t) of a drive h_e = p f(t)
    double he[3], hd[3];
    c->drive.eval(t, he, hd);
    return pp > 0.0 ? (hd[0] * pv[0] + hd[1] * pv[1] + hd[2] * pv[2]) / pp : 0.0;
  };
  T* warm = wsp<T>(c, c->off_warm);
  const size_t wb = 3 * c->nodes * sizeof(T);

  // Segment seg's states: y_m (checkpoint for m = 0, tape after), k1_m.
  auto seg_len = [&](int seg) { return std::min(steps, (seg + 1) * every) - seg * every; };
  auto yp = [&](int seg, int m) {
    return m == 0 ? R.cp(seg, 0) : (m < seg_len(seg) ? R.tape(m, 0) : R.yend());
  };
  auto k1p = [&](int seg, int m) { return m == 0 ? R.cp(seg, 1) : R.tape(m, 1); };
  T* k3tmp = R.vec(8);
  // Steps of one segment from its checkpoint into the tape, with the
  // current density of each stage state (same arithmetic as the forward);
  // the context's warm start must be that of the checkpoint.
  auto record = [&](int seg) -> scfft_status {
    const int s0 = seg * every, len = seg_len(seg);
    double t = t_of(s0);
    for (int m = 0; m < len; ++m) {
      const double h = t_of(s0 + m + 1) - t;
      ADJCHK(R.rhs(t + 0.5 * h, yp(seg, m), k1p(seg, m), 0.5 * h, R.tape(m, 2), R.tape(m, 3)));
      ADJCHK(R.rhs(t + 0.75 * h, yp(seg, m), R.tape(m, 2), 0.75 * h, k3tmp, R.tape(m, 4)));
      ADJCHK(R.combo(yp(seg, m + 1), yp(seg, m), k1p(seg, m), h * (2.0 / 9.0), R.tape(m, 2),
                     h * (1.0 / 3.0), k3tmp, h * (4.0 / 9.0)));
      if (m + 1 < len)
        ADJCHK(R.rhs(t + h, yp(seg, m + 1), nullptr, 0.0, R.tape(m + 1, 1), R.tape(m, 5)));
      t = t_of(s0 + m + 1);
    }
    return SCFFT_OK;
  };
  const int last = R.L.nseg - 1;

  // ---- forward: checkpoint at the start of every segment; the last segment
  // goes straight into the tape (it is reversed first) ----
  {
    T *Y = R.vec(0), *Y1 = R.vec(1), *K1 = R.vec(2), *K2 = R.vec(3), *K3 = R.vec(4), *K4 = R.vec(5);
    c->has_warm = false;
    ADJCHK(R.copy(Y, h0));
    ADJCHK(R.rhs(t0, Y, nullptr, 0.0, K1));
    double t = t0;
    for (int s = 0; s <= last * every; ++s) {
      if (s % every == 0) {
        const int seg = s / every;
        ADJCHK(R.copy(R.cp(seg, 0), Y));
        ADJCHK(R.copy(R.cp(seg, 1), K1));
        HIPCHK(c, hipMemcpyAsync(R.cp(seg, 2), warm, wb, hipMemcpyDeviceToDevice, c->stream));
      }
      if (s == last * every) break;
      const double h = t_of(s + 1) - t;
      ADJCHK(R.rhs(t + 0.5 * h, Y, K1, 0.5 * h, K2));
      ADJCHK(R.rhs(t + 0.75 * h, Y, K2, 0.75 * h, K3));
      ADJCHK(R.combo(Y1, Y, K1, h * (2.0 / 9.0), K2, h * (1.0 / 3.0), K3, h * (4.0 / 9.0)));
      ADJCHK(R.rhs(t + h, Y1, nullptr, 0.0, K4));
      std::swap(Y, Y1);
      std::swap(K1, K4);
      t = t_of(s + 1);
    }
    ADJCHK(record(last));
    if (hT) ADJCHK(R.copy(hT, R.yend()));
  }

  // ---- reverse ----
  T *ybar = R.vec(0), *k1n = R.vec(1), *wbA = R.vec(2), *wbB = R.vec(3), *k1b = R.vec(4),
    *k2b = R.vec(5), *k3b = R.vec(6), *ub = R.vec(7);
  double* sc = wsp<double>(c, c->off_adjs);
  HIPCHK(c, launch_zero_doubles(sc, 4, c->stream));
  ADJCHK(R.copy(ybar, hT_bar));
  ADJCHK(R.combo(k1n, nullptr, nullptr, 0.0, nullptr, 0.0, nullptr, 0.0));   // zero
  ADJCHK(R.combo(wbA, nullptr, nullptr, 0.0, nullptr, 0.0, nullptr, 0.0));
  for (int seg = last; seg >= 0; --seg) {
    const int s0 = seg * every, len = seg_len(seg);
    if (seg != last) {  // recompute the segment from its checkpoint
      HIPCHK(c, hipMemcpyAsync(warm, R.cp(seg, 2), wb, hipMemcpyDeviceToDevice, c->stream));
      c->has_warm = true;
      ADJCHK(record(seg));
    }
    // adjoint steps, last first
    for (int m = len - 1; m >= 0; --m) {
      const double ts = t_of(s0 + m), h = t_of(s0 + m + 1) - ts;
      // k4 = f(t + h, y_{n+1}; w3): cotangent k1n (the next step's k1), warm cotangent wbA
      ADJCHK(rhs_vjp_impl<T>(c, yp(seg, m + 1), nullptr, 0.0, true, k1n, wbA, ub, wbB, kbar, sc,
                             rate(ts + h), m + 1 < len ? R.tape(m, 5) : nullptr));
      ADJCHK(R.combo(ybar, ybar, ub, 1.0, nullptr, 0.0, nullptr, 0.0));
      // y_{n+1} = y + h (2/9 k1 + 1/3 k2 + 4/9 k3)
      ADJCHK(R.combo(k1b, nullptr, ybar, h * (2.0 / 9.0), nullptr, 0.0, nullptr, 0.0));
      ADJCHK(R.combo(k2b, nullptr, ybar, h * (1.0 / 3.0), nullptr, 0.0, nullptr, 0.0));
      ADJCHK(R.combo(k3b, nullptr, ybar, h * (4.0 / 9.0), nullptr, 0.0, nullptr, 0.0));
      // k3 = f(t + 3h/4, y + 3h/4 k2; w2)
      ADJCHK(rhs_vjp_impl<T>(c, yp(seg, m), R.tape(m, 2), 0.75 * h, true, k3b, wbB, ub, wbA, kbar, sc,
                             rate(ts + 0.75 * h), R.tape(m, 4)));
      ADJCHK(R.combo(ybar, ybar, ub, 1.0, nullptr, 0.0, nullptr, 0.0));
      ADJCHK(R.combo(k2b, k2b, ub, 0.75 * h, nullptr, 0.0, nullptr, 0.0));
      // k2 = f(t + h/2, y + h/2 k1; w1)
      ADJCHK(rhs_vjp_impl<T>(c, yp(seg, m), k1p(seg, m), 0.5 * h, true, k2b, wbA, ub, wbB, kbar, sc,
                             rate(ts + 0.5 * h), R.tape(m, 3)));
      ADJCHK(R.combo(ybar, ybar, ub, 1.0, nullptr, 0.0, nullptr, 0.0));
      ADJCHK(R.combo(k1n, k1b, ub, 0.5 * h, nullptr, 0.0, nullptr, 0.0));
      std::swap(wbA, wbB);
    }
  }
  // the first evaluation k1 = f(t0, y0) started without a warm start
  ADJCHK(rhs_vjp_impl<T>(c, h0, nullptr, 0.0, false, k1n, wbA, ub, nullptr, kbar, sc, rate(t0)));
  ADJCHK(R.combo(h0_bar, ybar, ub, 1.0, nullptr, 0.0, nullptr, 0.0));
  double r[4];
  HIPCHK(c, hipMemcpyAsync(r, sc, sizeof r, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (n_bar) *n_bar = r[0];
  if (p_bar)
    for (int d = 0; d < 3; ++d) p_bar[d] = r[1 + d];
  c->has_warm = false;  // the context's warm start no longer belongs to a caller's trajectory
  return SCFFT_OK;
}

// ---------------------------------------------------------------------------
// graph-replayed fixed-step integration
// ---------------------------------------------------------------------------
// Caller workspace: the device state of the replays, the error norm of each
// step and the table of applied-field rates (3 stages x 3 components per step).
struct GraphLayout {
  size_t off_state = 0, off_err = 0, off_hist = 0, off_tab = 0, off_mhist = 0, total = 0;
};

GraphLayout graph_layout(int steps) {
  GraphLayout L;
  size_t o = 0;
  L.off_state = o;  o = align_up(o + sizeof(GraphState));
  L.off_err = o;    o = align_up(o + sizeof(double));
  L.off_hist = o;   o = align_up(o + (size_t)steps * sizeof(double));
  L.off_tab = o;    o = align_up(o + (size_t)steps * 9 * sizeof(double));
  L.off_mhist = o;  o = align_up(o + (size_t)steps * 6 * sizeof(double));
  L.total = o;
  return L;
}

// One Bogacki-Shampine step as launched while a graph is captured: the
// three right-hand sides read their applied-field rate from row *step of the
// table, and every kernel returns at once after the stop flag is set.
template <typename T>
scfft_status graph_step(scfft_ctx* c, T* const r[6], double dt, GraphState* gs, double* err,
                        double* hist, double* mhist) {
  const double thr = 1e-6 / 2e-4;  // atol / rtol of the default controller
  scfft_status st;
  c->g_hedot_stage = 0;
  if ((st = rhs_impl<T>(c, 0.0, r[B_Y], r[B_K2], nullptr, r[B_K1], 0.5 * dt)) < 0) return st;
  c->g_hedot_stage = 1;
  if ((st = rhs_impl<T>(c, 0.0, r[B_Y], r[B_K3], nullptr, r[B_K2], 0.75 * dt)) < 0) return st;
  HIPCHK(c, launch_combo<T>(r[B_Y1], r[B_Y], r[B_K1], dt * (2.0 / 9.0), r[B_K2], dt * (1.0 / 3.0),
                            r[B_K3], dt * (4.0 / 9.0), 3 * c->nodes, c->stream, &gs->stop));
  c->g_hedot_stage = 2;
  // the FSAL evaluation at the new state also sums its moment (power-law pass)
  double* mom = wsp<double>(c, c->off_mom);
  if ((st = rhs_impl<T>(c, 0.0, r[B_Y1], r[B_K4], nullptr, nullptr, 0.0, mom)) < 0) return st;
  const int xbm = xpass_blocks<T>(make_plan<T>(c));
  HIPCHK(c, launch_graph_moment(mom, xbm, gs, mhist, c->stream));
  double* part = wsp<double>(c, c->off_part);
  HIPCHK(c, launch_errnorm<T>(r[B_Y], r[B_Y1], r[B_K1], r[B_K2], r[B_K3], r[B_K4], dt, thr,
                              3 * c->nodes, part, kReduceBlocks, c->stream, &gs->stop));
  HIPCHK(c, launch_max_partials(part, kReduceBlocks, err, c->stream, &gs->stop));
  HIPCHK(c, launch_graph_step_end(err, gs, hist, c->stream));
  return SCFFT_OK;
}

template <typename T>
scfft_status graph_begin_impl(scfft_ctx* c, double t0, double t1, int steps, T* h, char* gws) {
  const size_t fb = 3 * c->nodes * sizeof(T);
  T* buf[6];
  for (int k = 0; k < 6; ++k) buf[k] = wsp<T>(c, c->off_ode + (size_t)k * fb);
  const double dt = (t1 - t0) / steps;
  const GraphLayout L = graph_layout(steps);
  GraphState* gs = reinterpret_cast<GraphState*>(gws + L.off_state);
  double* err = reinterpret_cast<double*>(gws + L.off_err);
  double* hist = reinterpret_cast<double*>(gws + L.off_hist);
  double* tab = reinterpret_cast<double*>(gws + L.off_tab);
  double* mhist = reinterpret_cast<double*>(gws + L.off_mhist);
  // applied-field rates at the stage times of every step, evaluated on the host
  c->graph_hedot.assign((size_t)steps * 9, 0.0);
  const double frac[3] = {0.5, 0.75, 1.0};
  for (int s = 0; s < steps; ++s) {
    const double ts = t0 + s * dt;
    for (int q = 0; q < 3; ++q) {
      double he[3], hd[3];
      c->drive.eval(ts + frac[q] * dt, he, hd);
      for (int d = 0; d < 3; ++d) c->graph_hedot[(size_t)s * 9 + q * 3 + d] = hd[d];
    }
  }
  c->graph_accepted = -1;
  HIPCHK(c, hipMemcpyAsync(tab, c->graph_hedot.data(), c->graph_hedot.size() * sizeof(double),
                           hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, launch_graph_reset(gs, c->stream));
  // initial state and its rate (plain launches)
  HIPCHK(c, hipMemcpyAsync(buf[B_Y], h, fb, hipMemcpyDeviceToDevice, c->stream));
  scfft_status st = rhs_impl<T>(c, t0, buf[B_Y], buf[B_K1], nullptr);
  if (st < 0) return st;
  // capture one step for each parity of the buffer roles (accepting a step
  // swaps Y/Y1, K1/K4), unless the graphs of the last integration still fit:
  // chunks of equal length give step sizes equal up to the rounding of
  // (t1 - t0) / steps, and the captured step size is kept
  const bool cached = c->graph_exec[0] && c->graph_exec[1] && c->graph_key.gws == gws &&
                      c->graph_key.steps == steps && c->graph_key.epoch == c->epoch &&
                      std::fabs(c->graph_key.dt - dt) <= 1e-12 * std::fabs(dt);
  st = SCFFT_OK;
  if (!cached) {
    for (auto& x : c->graph_exec)
      if (x) (void)hipGraphExecDestroy(x), x = nullptr;
    c->graph_key.epoch = 0;
    hipStream_t cs = nullptr;
    HIPCHK(c, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    const hipStream_t saved = c->stream;
    const bool saved_prof = c->prof;
    c->stream = cs;
    c->prof = false;
    c->graph_stop = &gs->stop;
    c->g_hedot_tab = tab;
    c->g_hedot_step = &gs->step;
    T* r[6];
    for (int k = 0; k < 6; ++k) r[k] = buf[k];
    for (int par = 0; par < 2 && st == SCFFT_OK; ++par) {
      hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
      if (e != hipSuccess) {
        st = fail(c, SCFFT_ERR_DEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
        break;
      }
      const scfft_status sst = graph_step<T>(c, r, dt, gs, err, hist, mhist);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(cs, &g);
      if (sst < 0) {
        st = sst;
      } else if (e != hipSuccess) {
        st = fail(c, SCFFT_ERR_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
      } else {
        e = hipGraphInstantiate(&c->graph_exec[par], g, nullptr, nullptr, 0);
        if (e != hipSuccess) st = fail(c, SCFFT_ERR_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
      }
      if (g) (void)hipGraphDestroy(g);
      std::swap(r[B_Y], r[B_Y1]);
      std::swap(r[B_K1], r[B_K4]);
    }
    c->stream = saved;
    c->prof = saved_prof;
    c->graph_stop = nullptr;
    c->g_hedot_tab = nullptr;
    c->g_hedot_step = nullptr;
    c->g_hedot_stage = 0;
    (void)hipStreamDestroy(cs);
    if (st == SCFFT_OK) {
      c->graph_key.gws = gws;
      c->graph_key.steps = steps;
      c->graph_key.dt = dt;
      c->graph_key.epoch = c->epoch;
    }
  }
  if (st == SCFFT_OK) {
    for (int s = 0; s < steps; ++s) {
      const hipError_t e = hipGraphLaunch(c->graph_exec[s & 1], c->stream);
      if (e != hipSuccess) {
        st = fail(c, SCFFT_ERR_DEVICE, "hipGraphLaunch: %s", hipGetErrorString(e));
        break;
      }
    }
  }
  if (st != SCFFT_OK) {
    (void)hipStreamSynchronize(c->stream);
    for (auto& x : c->graph_exec)
      if (x) (void)hipGraphExecDestroy(x), x = nullptr;
    c->graph_key.epoch = 0;
    return st;
  }
  c->graph_busy = true;
  c->graph_ws = gws;
  c->graph_steps = steps;
  c->graph_t0 = t0;
  c->graph_dt = dt;
  c->graph_h = h;
  return SCFFT_OK;
}

template <typename T>
scfft_status graph_wait_impl(scfft_ctx* c, scfft_ode_stats* stats) {
  const GraphLayout L = graph_layout(c->graph_steps);
  GraphState hs{0, 0, -1, 0};
  hipError_t e = hipMemcpyAsync(&hs, c->graph_ws + L.off_state, sizeof hs, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  c->graph_busy = false;
  if (e != hipSuccess) return fail(c, SCFFT_ERR_DEVICE, "graph integration: %s", hipGetErrorString(e));
  // the last accepted state is in the Y buffer of the parity of the next (or failed) step
  const size_t fb = 3 * c->nodes * sizeof(T);
  const int next = hs.bad >= 0 ? hs.bad : hs.step;
  const int slot = (next & 1) ? B_Y1 : B_Y;
  HIPCHK(c, hipMemcpyAsync(c->graph_h, wsp<char>(c, c->off_ode + (size_t)slot * fb), fb,
                           hipMemcpyDeviceToDevice, c->stream));
  double err_last = 0.0;
  const int last = hs.bad >= 0 ? hs.bad : hs.step - 1;
  if (last >= 0)
    HIPCHK(c, hipMemcpyAsync(&err_last, c->graph_ws + L.off_hist + (size_t)last * sizeof(double),
                             sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->graph_accepted = hs.step;
  if (stats) {
    std::memset(stats, 0, sizeof *stats);
    stats->accepted = hs.step;
    stats->rhs_calls = 1 + 3 * (int64_t)(hs.step + (hs.bad >= 0 ? 1 : 0));
    stats->iters_total = stats->rhs_calls * c->opts.fixed_iter;
    stats->t_s = (hs.step == c->graph_steps ? c->graph_t0 + c->graph_steps * c->graph_dt
                                            : c->graph_t0 + hs.step * c->graph_dt) * c->u.t0;
    stats->dt_last_s = c->graph_dt * c->u.t0;
    stats->err_last = err_last;
  }
  return hs.bad >= 0 ? fail(c, SCFFT_ERR_NAN, "non-finite error norm at step %d", hs.bad) : SCFFT_OK;
}

// Autotuner over the pass schedules of one right-hand-side call: times each
// candidate on the caller's state with HIP events on the context stream and
// keeps the faster (rhs option fuse_xy).  The warm start is saved in an ODE
// buffer and restored after every timed run.
template <typename T>
scfft_status autotune_impl(scfft_ctx* c, const T* h, int calls, int* choice, double* ms_best) {
  const Plan<T> p = make_plan<T>(c);
  // (fuse_xy, x_alt, y_alt, z_alt): row/column passes with either element
  // count of the per-component x passes, and the fused plane pass where it
  // fits (which has no per-component x pass to vary), each with either
  // element count of the y and z passes
  struct Cand {
    int fuse, x, y, z;
  };
  std::vector<Cand> cand;
  for (int y = 0; y < 2; ++y)
    for (int z = 0; z < 2; ++z) {
      cand.push_back({0, 0, y, z});
      cand.push_back({0, 1, y, z});
      if (xypass_supported<T>(p)) cand.push_back({2, 0, y, z});
    }
  const size_t fb = 3 * c->nodes * sizeof(T);
  T* out = wsp<T>(c, c->off_ode + 4 * fb);
  T* saved = wsp<T>(c, c->off_ode + 5 * fb);
  const bool had_warm = c->has_warm;
  if (had_warm) HIPCHK(c, hipMemcpyAsync(saved, wsp<T>(c, c->off_warm), fb, hipMemcpyDeviceToDevice, c->stream));
  auto restore = [&]() -> hipError_t {
    c->has_warm = had_warm;
    return had_warm ? hipMemcpyAsync(wsp<T>(c, c->off_warm), saved, fb, hipMemcpyDeviceToDevice, c->stream)
                    : hipSuccess;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(c, hipEventCreate(&e0));
  hipError_t he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(c, SCFFT_ERR_DEVICE, "hipEventCreate: %s", hipGetErrorString(he));
  }
  const scfft_rhs_opts keep = c->opts;
  scfft_status st = SCFFT_OK;
  double best = INFINITY;
  Cand pick{keep.fuse_xy, keep.x_alt, keep.y_alt, keep.z_alt};
  for (const auto& fa : cand) {
    c->opts.fuse_xy = fa.fuse;
    c->opts.x_alt = fa.x;
    c->opts.y_alt = fa.y;
    c->opts.z_alt = fa.z;
    if ((he = restore()) != hipSuccess) break;
    if ((st = rhs_impl<T>(c, 0.0, h, out, nullptr)) < 0) break;          // warm-up
    if ((he = hipEventRecord(e0, c->stream)) != hipSuccess) break;
    for (int k = 0; k < calls && st >= 0; ++k) st = rhs_impl<T>(c, 0.0, h, out, nullptr);
    if (st < 0) break;
    if ((he = hipEventRecord(e1, c->stream)) != hipSuccess) break;
    if ((he = hipEventSynchronize(e1)) != hipSuccess) break;
    float ms = 0.0f;
    if ((he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
    if (ms / calls < best) {
      best = ms / calls;
      pick = fa;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->opts = keep;
  if (st < 0) return st;
  if (he != hipSuccess) return fail(c, SCFFT_ERR_DEVICE, "autotune: %s", hipGetErrorString(he));
  HIPCHK(c, restore());
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->opts.fuse_xy = pick.fuse;
  c->opts.x_alt = pick.x;
  c->opts.y_alt = pick.y;
  c->opts.z_alt = pick.z;
  ++c->epoch;
  if (choice) *choice = pick.fuse;
  if (ms_best) *ms_best = best;
  return SCFFT_OK;
}

template <typename T>
scfft_status region_impl(scfft_ctx* c, const T* h, const uint8_t* region, double* b) {
  double* part = wsp<double>(c, c->off_part);
  double* out = wsp<double>(c, c->off_scal);
  HIPCHK(c, launch_region_abs<T>(h, region, c->nodes, part, kReduceBlocks, c->stream));
  HIPCHK(c, launch_sum_partials(part, kReduceBlocks, 2, 2, out, c->stream));
  double r[2];
  HIPCHK(c, hipMemcpyAsync(r, out, sizeof r, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *b = r[1] > 0 ? r[0] / r[1] * c->u.h_scale * kMu0 : 0.0;
  return SCFFT_OK;
}

// ||(1 - chi) j|| / ||chi j|| with j = C_s h (Eq. 4) formed in the reverse-mode
// buffer (free outside reverse-mode calls).
template <typename T>
scfft_status stray_impl(scfft_ctx* c, const T* h, double* frac) {
  T* j = wsp<T>(c, c->off_adj);
  scfft_status st = apply_operator<T>(c, h, j, Z_CURL, 1.0);
  if (st < 0) return st;
  double* part = wsp<double>(c, c->off_part);
  double* out = wsp<double>(c, c->off_scal);
  HIPCHK(c, launch_mask_sq<T>(j, wsp<uint8_t>(c, c->off_chi), c->nodes, part, kReduceBlocks, c->stream));
  HIPCHK(c, launch_sum_partials(part, kReduceBlocks, 2, 2, out, c->stream));
  double r[2];
  HIPCHK(c, hipMemcpyAsync(r, out, sizeof r, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *frac = r[1] > 0.0 ? std::sqrt(r[0] / r[1]) : 0.0;
  return SCFFT_OK;
}

template <typename T>
scfft_status probe_impl(scfft_ctx* c, const T* h, const double* xyz, int npts, double* b) {
  double* dpts = wsp<double>(c, c->off_probe);
  double* dout = dpts + 3 * kProbeChunk;
  std::vector<double> pts;
  for (int p0 = 0; p0 < npts; p0 += kProbeChunk) {
    const int np = std::min(kProbeChunk, npts - p0);
    pts.assign(xyz + 3 * (size_t)p0, xyz + 3 * (size_t)(p0 + np));
    for (double& v : pts) v /= c->u.l;
    HIPCHK(c, hipMemcpyAsync(dpts, pts.data(), pts.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_probe<T>(h, c->n[0], c->n[1], c->n[2], dpts, np, -c->L[0] + 0.5 * c->h[0],
                              -c->L[1] + 0.5 * c->h[1], -c->L[2] + 0.5 * c->h[2], c->h[0], c->h[1],
                              c->h[2], dout, c->stream));
    HIPCHK(c, hipMemcpyAsync(b + 3 * (size_t)p0, dout, 3 * (size_t)np * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  const double s = c->u.h_scale * kMu0;
  for (int i = 0; i < 3 * npts; ++i) b[i] *= s;
  return SCFFT_OK;
}

scfft_status set_mask_host(scfft_ctx* c, const std::vector<uint8_t>& m) {
  HIPCHK(c, hipMemcpyAsync(wsp<uint8_t>(c, c->off_chi), m.data(), c->nodes, hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  int64_t in = 0;
  int lo[3] = {c->n[0], c->n[1], c->n[2]}, hi[3] = {0, 0, 0};
  for (int z = 0; z < c->n[2]; ++z)
    for (int y = 0; y < c->n[1]; ++y)
      for (int x = 0; x < c->n[0]; ++x)
        if (m[((size_t)z * c->n[1] + y) * c->n[0] + x]) {
          ++in;
          const int id[3] = {x, y, z};
          for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], id[a]);
            hi[a] = std::max(hi[a], id[a] + 1);
          }
        }
  for (int a = 0; a < 3; ++a) {
    c->box_lo[a] = in ? lo[a] : 0;
    c->box_hi[a] = in ? hi[a] : 0;
  }
  c->n_in = in;
  c->n_out = (int64_t)c->nodes - in;
  c->has_mask = true;
  c->has_warm = false;
  drop_cont(c);
  ++c->epoch;
  mask_betti(c->n, m.data(), c->betti);
  return c->betti[1] > 0 ? SCFFT_WARN_TOPOLOGY : SCFFT_OK;
}

template <typename T>
scfft_status upload_tables(scfft_ctx* c) {
  std::vector<char> t = build_tables<T>(c);
  HIPCHK(c, hipMemcpyAsync(c->ws + c->off_tab, t.data(), t.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemsetAsync(c->ws + c->off_clamp, 0, sizeof(unsigned long long), c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->clamp_seen = 0;
  return SCFFT_OK;
}

struct StateHeader {
  uint64_t magic;
  int32_t version, prec, n[3], has_warm;
  scfft_rhs_opts opts;
  uint64_t warm_bytes;
  // version 2: the adaptive iteration's first launch count and the
  // continuation of the adaptive step controller (k1 follows the warm start)
  int32_t iter_guess, cont_valid, cont_rejected, cont_has_k1;
  double cont_t, cont_dt;
  uint64_t k1_bytes;
};
const uint64_t kStateMagic = 0x5343464654535431ull;  // "SCFFTST1"

}  // namespace

// ===========================================================================
// batches of same-size instances
// ===========================================================================
// A batch advances several contexts of one grid together: every pass is one
// launch over all of them (instance = blockIdx.z), so small boxes fill the
// chip.  The members' workspaces lie at a constant stride in one allocation,
// so instance b's buffers are instance 0's shifted by b strides; the
// per-instance scalars (n, rho_out, stage coefficients, applied-field rates)
// sit in each member's BPar slot, uploaded from pinned host rows.
constexpr int kBatchRing = 4;       // pinned row sets in flight (plain batched calls)
constexpr int kMaxBatch = 512;      // members per batch (their BPar rows fit the probe area)

struct scfft_batch {
  std::vector<scfft_ctx*> m;
  size_t stride = 0;                          // bytes from one member's workspace to the next
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};   // box holding Omega of every member
  double* pin = nullptr;                      // kBatchRing sets of BPar rows, one row per member
  hipEvent_t ev[kBatchRing] = {};
  bool ev_live[kBatchRing] = {};
  int ring = 0;
  // graph-replayed fixed steps
  bool busy = false;
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  char* gws = nullptr;
  int steps = 0;
  double t0_s = 0.0, t1_s = 0.0;
  void* h = nullptr;
  int64_t fstride = 0;
  std::vector<double> tab;                    // host rate tables (alive until the wait)
};

namespace {

struct BatchGraphLayout {
  size_t off_state = 0, off_hist = 0, off_tab = 0, total = 0;
};

// graph workspace of a batch: replay state, error norms [member][step], rate
// tables [member][step][stage][component]
BatchGraphLayout batch_graph_layout(int count, int steps) {
  BatchGraphLayout L;
  size_t o = 0;
  L.off_state = o;  o = align_up(o + sizeof(GraphState));
  L.off_hist = o;   o = align_up(o + (size_t)count * steps * sizeof(double));
  L.off_tab = o;    o = align_up(o + (size_t)count * steps * 9 * sizeof(double));
  L.total = o;
  return L;
}

// The next set of pinned rows (waits until its last upload has been read),
// filled with each member's n and rho_out.
scfft_status batch_rows(scfft_batch* B, double** rows) {
  scfft_ctx* c = B->m[0];
  const int k = B->ring;
  if (B->ev_live[k]) HIPCHK(c, hipEventSynchronize(B->ev[k]));
  double* r = B->pin + (size_t)k * B->m.size() * kBParDoubles;
  std::memset(r, 0, B->m.size() * kBParDoubles * sizeof(double));
  for (size_t b = 0; b < B->m.size(); ++b) {
    r[b * kBParDoubles + BP_N] = B->m[b]->mat.n_power;
    r[b * kBParDoubles + BP_RHO] = B->m[b]->mat.rho_out;
  }
  *rows = r;
  return SCFFT_OK;
}

// upload the rows of batch_rows (one copy into member 0's probe area) and
// scatter them into every member's BPar slot
scfft_status batch_upload(scfft_batch* B, const double* rows) {
  scfft_ctx* c = B->m[0];
  double* stage = wsp<double>(c, c->off_probe);
  HIPCHK(c, hipMemcpyAsync(stage, rows, B->m.size() * kBParDoubles * sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, hipEventRecord(B->ev[B->ring], c->stream));
  HIPCHK(c, launch_strided_copy<double>(wsp<double>(c, c->off_bpar), (int64_t)B->stride, stage,
                                        kBParDoubles * (int64_t)sizeof(double), kBParDoubles, (int)B->m.size(),
                                        c->stream));
  B->ev_live[B->ring] = true;
  B->ring = (B->ring + 1) % kBatchRing;
  return SCFFT_OK;
}

bool batch_warm(const scfft_batch* B, scfft_status* st) {
  for (auto* m : B->m)
    if (m->has_warm != B->m[0]->has_warm) {
      *st = fail(B->m[0], SCFFT_ERR_STATE, "batch members differ in having a warm start");
      return false;
    }
  return true;
}

// One right-hand side (fixed iteration count) of every member as batched
// launches.  Instance b reads h + b zs_in bytes (plus in2_coef in2 of its
// own, in2_sel: BPar stage coefficient) and writes hdot + b zs_out bytes; its
// applied-field rate is tab[b zs_tab bytes + 9 *step + 3 stage + c].
template <typename T>
scfft_status batch_rhs_passes(scfft_batch* B, const T* h, T* hdot, int64_t zs_in, int64_t zs_out,
                              const T* in2, int in2_sel, const double* tab, int64_t zs_tab,
                              const int* step, int stage) {
  scfft_ctx* c = B->m[0];
  Plan<T> p = make_plan<T>(c);
  p.batch = (int)B->m.size();
  p.zs_main = (int64_t)(B->stride / sizeof(C2<T>));
  XArgs<T> a = base_args<T>(c);
  a.zs_ws = (int64_t)B->stride;
  a.zs_in = zs_in;
  a.zs_out = zs_out;
  a.zpar = wsp<double>(c, c->off_bpar);
  a.in2 = in2;
  a.in2_sel = in2 ? in2_sel : -1;
  a.hedot_tab = tab;
  a.zs_tab = zs_tab;
  a.hedot_step = step;
  a.hedot_stage = stage;
  const scfft_status st =
      rhs_fixed_passes<T>(c, p, a, c->has_warm, wsp<T>(c, c->off_warm), B->lo, B->hi, h, hdot);
  if (st < 0) return st;
  for (auto* m : B->m) {
    m->has_warm = true;
    drop_cont(m);
  }
  return SCFFT_OK;
}

template <typename T>
scfft_status batch_rhs_impl(scfft_batch* B, double t_s, const T* h, T* hdot, int64_t fstride) {
  scfft_ctx* c = B->m[0];
  scfft_status st;
  if (!batch_warm(B, &st)) return st;
  double* rows = nullptr;
  if ((st = batch_rows(B, &rows)) < 0) return st;
  for (size_t b = 0; b < B->m.size(); ++b) {
    double he[3], hd[3];
    B->m[b]->drive.eval(t_s / B->m[b]->u.t0, he, hd);
    for (int d = 0; d < 3; ++d) rows[b * kBParDoubles + BP_HEDOT + d] = hd[d];
  }
  if ((st = batch_upload(B, rows)) < 0) return st;
  double* par = wsp<double>(c, c->off_bpar);
  const int64_t fs = fstride * (int64_t)sizeof(T);
  return batch_rhs_passes<T>(B, h, hdot, fs, fs, nullptr, -1, par + BP_HEDOT, (int64_t)B->stride,
                             reinterpret_cast<const int*>(par + BP_ZERO), 0);
}

// One Bogacki-Shampine step of every member as batched launches, as captured
// in a graph (the steps of graph_step, with per-member step sizes, stage
// coefficients and rate tables).
template <typename T>
scfft_status batch_graph_step(scfft_batch* B, T* const r[6], GraphState* gs, const double* tab, int steps,
                              double* hist) {
  scfft_ctx* c = B->m[0];
  const int count = (int)B->m.size();
  const int64_t zs = (int64_t)B->stride;
  const int64_t zt = (int64_t)steps * 9 * (int64_t)sizeof(double);
  double* par = wsp<double>(c, c->off_bpar);
  const double thr = 1e-6 / 2e-4;  // atol / rtol of the default controller
  scfft_status st;
  if ((st = batch_rhs_passes<T>(B, r[B_Y], r[B_K2], zs, zs, r[B_K1], BP_C2 - 2, tab, zt, &gs->step, 0)) < 0)
    return st;
  if ((st = batch_rhs_passes<T>(B, r[B_Y], r[B_K3], zs, zs, r[B_K2], BP_C3 - 2, tab, zt, &gs->step, 1)) < 0)
    return st;
  HIPCHK(c, launch_combo_batch<T>(r[B_Y1], r[B_Y], r[B_K1], r[B_K2], r[B_K3], par, 3 * c->nodes, count, zs,
                                  c->stream, &gs->stop));
  if ((st = batch_rhs_passes<T>(B, r[B_Y1], r[B_K4], zs, zs, nullptr, -1, tab, zt, &gs->step, 2)) < 0)
    return st;
  double* part = wsp<double>(c, c->off_part);
  HIPCHK(c, launch_errnorm_batch<T>(r[B_Y], r[B_Y1], r[B_K1], r[B_K2], r[B_K3], r[B_K4], par, thr, 3 * c->nodes,
                                    part, kReduceBlocks, count, zs, c->stream, &gs->stop));
  HIPCHK(c, launch_max_partials_batch(part, kReduceBlocks, par + BP_ERR, count, zs, c->stream, &gs->stop));
  HIPCHK(c, launch_batch_step_end(par + BP_ERR, zs, count, steps, gs, hist, c->stream));
  return SCFFT_OK;
}

void batch_drop_graphs(scfft_batch* B) {
  for (auto& x : B->exec)
    if (x) (void)hipGraphExecDestroy(x), x = nullptr;
}

template <typename T>
scfft_status batch_graph_begin_impl(scfft_batch* B, double t0_s, double t1_s, int steps, char* gws, T* h,
                                    int64_t fstride) {
  scfft_ctx* c = B->m[0];
  const int count = (int)B->m.size();
  const size_t fb = 3 * c->nodes * sizeof(T);
  const int64_t zs = (int64_t)B->stride;
  const BatchGraphLayout L = batch_graph_layout(count, steps);
  GraphState* gs = reinterpret_cast<GraphState*>(gws + L.off_state);
  double* hist = reinterpret_cast<double*>(gws + L.off_hist);
  double* tab = reinterpret_cast<double*>(gws + L.off_tab);
  T* buf[6];
  for (int k = 0; k < 6; ++k) buf[k] = wsp<T>(c, c->off_ode + (size_t)k * fb);
  scfft_status st;
  double* rows = nullptr;
  if ((st = batch_rows(B, &rows)) < 0) return st;
  // per member: dimensionless step (t' = t / t0 of its own jc), stage
  // coefficients, the rate at t0 (first evaluation) and at every stage time
  B->tab.assign((size_t)count * steps * 9, 0.0);
  const double frac[3] = {0.5, 0.75, 1.0};
  for (int b = 0; b < count; ++b) {
    const scfft_ctx* m = B->m[b];
    // the step as graph_begin_impl forms it, so a member replays bit for bit
    // what its own context would
    const double t0 = t0_s / m->u.t0, t1 = t1_s / m->u.t0, dt = (t1 - t0) / steps;
    double* r = rows + (size_t)b * kBParDoubles;
    r[BP_C2] = 0.5 * dt;
    r[BP_C3] = 0.75 * dt;
    r[BP_B1] = dt * (2.0 / 9.0);
    r[BP_B2] = dt * (1.0 / 3.0);
    r[BP_B3] = dt * (4.0 / 9.0);
    r[BP_DT] = dt;
    double he[3], hd[3];
    m->drive.eval(t0, he, hd);
    for (int d = 0; d < 3; ++d) r[BP_HEDOT + d] = hd[d];
    for (int s = 0; s < steps; ++s)
      for (int q = 0; q < 3; ++q) {
        m->drive.eval(t0 + s * dt + frac[q] * dt, he, hd);
        for (int d = 0; d < 3; ++d) B->tab[((size_t)b * steps + s) * 9 + q * 3 + d] = hd[d];
      }
  }
  if ((st = batch_upload(B, rows)) < 0) return st;
  HIPCHK(c, hipMemcpyAsync(tab, B->tab.data(), B->tab.size() * sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
  HIPCHK(c, launch_graph_reset(gs, c->stream));
  // the members' states into their Y buffers, then their first rates (plain launches)
  HIPCHK(c, launch_strided_copy<T>(buf[B_Y], zs, h, fstride * (int64_t)sizeof(T), 3 * c->nodes, count,
                                   c->stream));
  double* par = wsp<double>(c, c->off_bpar);
  if ((st = batch_rhs_passes<T>(B, buf[B_Y], buf[B_K1], zs, zs, nullptr, -1, par + BP_HEDOT, zs,
                                reinterpret_cast<const int*>(par + BP_ZERO), 0)) < 0)
    return st;
  // one step captured for each parity of the buffer roles, then replayed
  batch_drop_graphs(B);
  hipStream_t cs = nullptr;
  HIPCHK(c, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  const hipStream_t saved = c->stream;
  const bool saved_prof = c->prof;
  c->stream = cs;
  c->prof = false;
  c->graph_stop = &gs->stop;
  T* r[6];
  for (int k = 0; k < 6; ++k) r[k] = buf[k];
  st = SCFFT_OK;
  for (int parity = 0; parity < 2 && st == SCFFT_OK; ++parity) {
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
      st = fail(c, SCFFT_ERR_DEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
      break;
    }
    const scfft_status sst = batch_graph_step<T>(B, r, gs, tab, steps, hist);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    if (sst < 0) {
      st = sst;
    } else if (e != hipSuccess) {
      st = fail(c, SCFFT_ERR_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    } else {
      e = hipGraphInstantiate(&B->exec[parity], g, nullptr, nullptr, 0);
      if (e != hipSuccess) st = fail(c, SCFFT_ERR_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    if (g) (void)hipGraphDestroy(g);
    std::swap(r[B_Y], r[B_Y1]);
    std::swap(r[B_K1], r[B_K4]);
  }
  c->stream = saved;
  c->prof = saved_prof;
  c->graph_stop = nullptr;
  (void)hipStreamDestroy(cs);
  for (int s = 0; s < steps && st == SCFFT_OK; ++s) {
    const hipError_t e = hipGraphLaunch(B->exec[s & 1], c->stream);
    if (e != hipSuccess) st = fail(c, SCFFT_ERR_DEVICE, "hipGraphLaunch: %s", hipGetErrorString(e));
  }
  if (st != SCFFT_OK) {
    (void)hipStreamSynchronize(c->stream);
    batch_drop_graphs(B);
    return st;
  }
  B->busy = true;
  for (auto* m : B->m) m->graph_busy = true;
  B->gws = gws;
  B->steps = steps;
  B->t0_s = t0_s;
  B->t1_s = t1_s;
  B->h = h;
  B->fstride = fstride;
  return SCFFT_OK;
}

template <typename T>
scfft_status batch_graph_wait_impl(scfft_batch* B, scfft_ode_stats* stats) {
  scfft_ctx* c = B->m[0];
  const int count = (int)B->m.size();
  const BatchGraphLayout L = batch_graph_layout(count, B->steps);
  GraphState hs{0, 0, -1, 0};
  hipError_t e = hipMemcpyAsync(&hs, B->gws + L.off_state, sizeof hs, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  B->busy = false;
  for (auto* m : B->m) m->graph_busy = false;
  if (e != hipSuccess) return fail(c, SCFFT_ERR_DEVICE, "batch graph integration: %s", hipGetErrorString(e));
  // the last accepted states sit in the Y buffers of the parity of the next (or failed) step
  const size_t fb = 3 * c->nodes * sizeof(T);
  const int next = hs.bad >= 0 ? hs.bad : hs.step;
  const int slot = (next & 1) ? B_Y1 : B_Y;
  HIPCHK(c, launch_strided_copy<T>(static_cast<T*>(B->h), B->fstride * (int64_t)sizeof(T),
                                   wsp<T>(c, c->off_ode + (size_t)slot * fb), (int64_t)B->stride, 3 * c->nodes,
                                   count, c->stream));
  std::vector<double> hist((size_t)count * B->steps, 0.0);
  HIPCHK(c, hipMemcpyAsync(hist.data(), B->gws + L.off_hist, hist.size() * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const int last = hs.bad >= 0 ? hs.bad : hs.step - 1;
  const double dts = (B->t1_s - B->t0_s) / B->steps;
  if (stats) {
    for (int b = 0; b < count; ++b) {
      scfft_ode_stats& st = stats[b];
      std::memset(&st, 0, sizeof st);
      st.accepted = hs.step;
      st.rhs_calls = 1 + 3 * (int64_t)(hs.step + (hs.bad >= 0 ? 1 : 0));
      st.iters_total = st.rhs_calls * B->m[b]->opts.fixed_iter;
      st.t_s = hs.step == B->steps ? B->t1_s : B->t0_s + hs.step * dts;
      st.dt_last_s = dts;
      st.err_last = last >= 0 ? hist[(size_t)b * B->steps + last] : 0.0;
    }
  }
  return hs.bad >= 0 ? fail(c, SCFFT_ERR_NAN, "non-finite error norm at step %d", hs.bad) : SCFFT_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void scfft_default_rhs_opts(scfft_rhs_opts* o) {
  if (!o) return;
  o->delta_it = 2e-5;
  o->min_iter = 1;
  o->max_iter = 200;
  o->fixed_iter = 0;
  o->smooth_phi = 0;
  o->sigma_scale = 1.0;
  o->fuse_xy = 1;
  o->prune_box = 1;
  o->x_alt = 0;
  o->y_alt = 0;
  o->z_alt = 0;
}

void scfft_default_ode_opts(scfft_ode_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->rtol = 2e-4;
  o->atol = 1e-6;
}

scfft_status scfft_units(const scfft_material* m, double* t0_s, double* h_scale) {
  const char* why = nullptr;
  if (!m || !t0_s || !h_scale || !validate_material(*m, &why)) return SCFFT_ERR_ARG;
  Units u = make_units(*m);
  *t0_s = u.t0;
  *h_scale = u.h_scale;
  return SCFFT_OK;
}

scfft_status scfft_drive_eval(const scfft_drive* d, const scfft_material* m, double t_s,
                              double he[3], double hedot[3]) {
  const char* why = nullptr;
  if (!d || !m || !he || !hedot || !validate_material(*m, &why)) return SCFFT_ERR_ARG;
  Units u = make_units(*m);
  Drive dr;
  if (!dr.set(*d, u, &why)) return SCFFT_ERR_ARG;
  dr.eval(t_s / u.t0, he, hedot);
  return SCFFT_OK;
}

scfft_status scfft_voxelize_host(const scfft_grid* g, const scfft_material* m,
                                 const scfft_shape* shapes, int32_t n_shapes, uint8_t* mask) {
  const char* why = nullptr;
  if (!g || !m || !mask || !validate_material(*m, &why) || !validate_shapes(shapes, n_shapes, &why))
    return SCFFT_ERR_ARG;
  double hw[3];
  for (int a = 0; a < 3; ++a) {
    if (g->n[a] < 2 || g->n[a] > 4096 || !(g->half_width_m[a] > 0.0)) return SCFFT_ERR_SHAPE;
    hw[a] = g->half_width_m[a] / m->l_char_m;
  }
  voxelize(g->n, hw, m->l_char_m, shapes, n_shapes, mask);
  return SCFFT_OK;
}

scfft_status scfft_mask_betti_host(const int32_t n[3], const uint8_t* mask, int64_t betti[3]) {
  if (!n || !mask || !betti) return SCFFT_ERR_ARG;
  for (int a = 0; a < 3; ++a)
    if (n[a] < 1) return SCFFT_ERR_SHAPE;
  if ((int64_t)n[0] * n[1] * n[2] >= (int64_t)INT32_MAX) return SCFFT_ERR_SHAPE;
  const int nn[3] = {n[0], n[1], n[2]};
  mask_betti(nn, mask, betti);
  return betti[1] > 0 ? SCFFT_WARN_TOPOLOGY : SCFFT_OK;
}

scfft_status scfft_bs23_host(int64_t n, double* y, double t0, double t1, scfft_host_rhs f,
                             void* user, const scfft_ode_opts* o, scfft_ode_stats* st) {
  if (n <= 0 || !y || !f || !valid_ode_opts(o) || !st || !(t1 > t0)) return SCFFT_ERR_ARG;
  std::memset(st, 0, sizeof *st);
  HostOps ops;
  ops.n = n;
  for (auto& v : ops.b) v.assign((size_t)n, 0.0);
  ops.y = y;
  ops.f = f;
  ops.user = user;
  std::vector<double> stops(o->breakpoints_s, o->breakpoints_s + o->n_bp);
  return bs23_run(ops, t0, t1, *o, stops, *st);
}

scfft_status scfft_create(scfft_ctx** out, const scfft_grid* g, const scfft_material* m,
                          scfft_precision prec, void* hip_stream) {
  if (!out || !g || !m) return SCFFT_ERR_ARG;
  *out = nullptr;
  const char* why = nullptr;
  if (!validate_material(*m, &why)) return SCFFT_ERR_ARG;
  if (prec != SCFFT_F64 && prec != SCFFT_F32) return SCFFT_ERR_ARG;
  for (int a = 0; a < 3; ++a) {
    if (!fft_length_supported(g->n[a])) return SCFFT_ERR_SHAPE;
    if (!(g->half_width_m[a] > 0.0) || !std::isfinite(g->half_width_m[a])) return SCFFT_ERR_ARG;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return SCFFT_ERR_DEVICE;
  char* scratch_dev = nullptr;  // device address of the allocation-free curl's array
  if (scratch_on(dev, &scratch_dev) != hipSuccess) return SCFFT_ERR_DEVICE;
  scfft_ctx* c = new scfft_ctx();
  c->grid = *g;
  c->mat = *m;
  c->prec = prec;
  c->stream = (hipStream_t)hip_stream;
  c->device = dev;
  c->nodes = 1;
  for (int a = 0; a < 3; ++a) {
    c->n[a] = g->n[a];
    c->nodes *= (size_t)g->n[a];
    c->L[a] = g->half_width_m[a] / m->l_char_m;
    c->h[a] = 2.0 * c->L[a] / g->n[a];
  }
  c->u = make_units(*m);
  scfft_default_rhs_opts(&c->opts);
  c->sigma = 0.5 * std::sqrt(c->h[0] * c->h[0] + c->h[1] * c->h[1] + c->h[2] * c->h[2]);
  c->wsize = prec == SCFFT_F64 ? sizeof(double) : sizeof(float);
  layout(c);
  *out = c;
  return SCFFT_OK;
}

void scfft_destroy(scfft_ctx* ctx) {
  if (!ctx) return;
  if (ctx->graph_busy) (void)hipStreamSynchronize(ctx->stream);
  for (auto& x : ctx->graph_exec)
    if (x) (void)hipGraphExecDestroy(x);
  for (auto& e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->rb_pin || ctx->rb_ev[0]) (void)hipStreamSynchronize(ctx->stream);
  for (auto& e : ctx->rb_ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->rb_pin) (void)hipHostFree(ctx->rb_pin);
  delete ctx;
}

scfft_status scfft_workspace_size(const scfft_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return SCFFT_ERR_ARG;
  *bytes = ctx->total;
  return SCFFT_OK;
}

scfft_status scfft_set_workspace(scfft_ctx* ctx, void* dev_ptr, size_t bytes) {
  if (!ctx) return SCFFT_ERR_ARG;
  if (ctx->graph_busy) return fail(ctx, SCFFT_ERR_STATE, "a graph integration is enqueued");
  ++ctx->epoch;
  if (!dev_ptr) return fail(ctx, SCFFT_ERR_WORKSPACE, "workspace pointer is NULL");
  if (bytes < ctx->total)
    return fail(ctx, SCFFT_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", bytes, ctx->total);
  if (((uintptr_t)dev_ptr) % kAlign)
    return fail(ctx, SCFFT_ERR_WORKSPACE, "workspace must be %zu-byte aligned", kAlign);
  ctx->ws = (char*)dev_ptr;
  ctx->ws_bytes = bytes;
  ctx->has_mask = ctx->has_kappa = ctx->has_warm = false;
  drop_cont(ctx);
  // the sigma of the context may have been rescaled by options; rebuild tables
  return ctx->prec == SCFFT_F64 ? upload_tables<double>(ctx) : upload_tables<float>(ctx);
}

scfft_status scfft_voxelize(scfft_ctx* ctx, const scfft_shape* shapes, int32_t n_shapes) {
  if (!ctx) return SCFFT_ERR_ARG;
  if (ctx->graph_busy) return fail(ctx, SCFFT_ERR_STATE, "a graph integration is enqueued");
  scfft_status st;
  if (!ready(ctx, false, &st)) return st;
  const char* why = nullptr;
  if (!validate_shapes(shapes, n_shapes, &why)) return fail(ctx, SCFFT_ERR_ARG, "%s", why);
  std::vector<uint8_t> m(ctx->nodes);
  voxelize(ctx->n, ctx->L, ctx->mat.l_char_m, shapes, n_shapes, m.data());
  return set_mask_host(ctx, m);
}

scfft_status scfft_set_mask(scfft_ctx* ctx, const uint8_t* dev_mask) {
  if (!ctx) return SCFFT_ERR_ARG;
  if (ctx->graph_busy) return fail(ctx, SCFFT_ERR_STATE, "a graph integration is enqueued");
  scfft_status st;
  if (!ready(ctx, false, &st)) return st;
  if (!dev_mask) return fail(ctx, SCFFT_ERR_ARG, "mask pointer is NULL");
  std::vector<uint8_t> m(ctx->nodes);
  HIPCHK(ctx, hipMemcpyAsync(m.data(), dev_mask, ctx->nodes, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return set_mask_host(ctx, m);
}

scfft_status scfft_set_jc_map(scfft_ctx* ctx, const void* dev_kappa) {
  if (!ctx) return SCFFT_ERR_ARG;
  if (ctx->graph_busy) return fail(ctx, SCFFT_ERR_STATE, "a graph integration is enqueued");
  ++ctx->epoch;
  scfft_status st;
  if (!ready(ctx, false, &st)) return st;
  if (!dev_kappa) {
    ctx->has_kappa = false;
    return SCFFT_OK;
  }
  drop_cont(ctx);
  ctx->has_kappa = false;
  HIPCHK(ctx, hipMemcpyAsync(ctx->ws + ctx->off_kappa, dev_kappa, ctx->nodes * ctx->wsize,
                             hipMemcpyDeviceToDevice, ctx->stream));
  // Eq. 1 uses ln kappa: every value must be finite and > 0
  double* part = wsp<double>(ctx, ctx->off_part);
  double* out = wsp<double>(ctx, ctx->off_scal);
  HIPCHK(ctx, ctx->prec == SCFFT_F64
                  ? launch_count_nonpositive<double>(wsp<double>(ctx, ctx->off_kappa), ctx->nodes, part,
                                                     kReduceBlocks, ctx->stream)
                  : launch_count_nonpositive<float>(wsp<float>(ctx, ctx->off_kappa), ctx->nodes, part,
                                                    kReduceBlocks, ctx->stream));
  HIPCHK(ctx, launch_sum_partials(part, kReduceBlocks, 1, 1, out, ctx->stream));
  double bad = 0.0;
  HIPCHK(ctx, hipMemcpyAsync(&bad, out, sizeof bad, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (bad > 0.0)
    return fail(ctx, SCFFT_ERR_ARG, "jc map: %.0f values are not finite and > 0", bad);
  ctx->has_kappa = true;
  return SCFFT_OK;
}

scfft_status scfft_set_drive(scfft_ctx* ctx, const scfft_drive* d) {
  if (!ctx || !d) return SCFFT_ERR_ARG;
  if (ctx->graph_busy) return fail(ctx, SCFFT_ERR_STATE, "a graph integration is enqueued");
  ++ctx->epoch;
  drop_cont(ctx);
  const char* why = nullptr;
  Drive dr;
  if (!dr.set(*d, ctx->u, &why)) return fail(ctx, SCFFT_ERR_ARG, "%s", why);
  ctx->drive = dr;
  ctx->has_drive = true;
  return SCFFT_OK;
}

scfft_status scfft_set_field_law(scfft_ctx* ctx, double b0_T, double alpha) {
  if (!ctx) return SCFFT_ERR_ARG;
  if (ctx->graph_busy) return fail(ctx, SCFFT_ERR_STATE, "a graph integration is enqueued");
  ++ctx->epoch;
  drop_cont(ctx);
  if (!(b0_T >= 0.0) || !(alpha >= 0.0) || !std::isfinite(b0_T) || !std::isfinite(alpha))
    return fail(ctx, SCFFT_ERR_ARG, "field law needs b0_T >= 0 and alpha >= 0");
  // |B| / B0 = mu0 h_scale |h'| / B0 with h' the dimensionless field (Eq. 8)
  ctx->field_hk_inv = b0_T > 0.0 ? kMu0 * ctx->u.h_scale / b0_T : 0.0;
  ctx->field_alpha = b0_T > 0.0 ? alpha : 0.0;
  return SCFFT_OK;
}

scfft_status scfft_set_anisotropy(scfft_ctx* ctx, const double a[3]) {
  if (!ctx) return SCFFT_ERR_ARG;
  if (ctx->graph_busy) return fail(ctx, SCFFT_ERR_STATE, "a graph integration is enqueued");
  ++ctx->epoch;
  drop_cont(ctx);
  if (a) {
    for (int d = 0; d < 3; ++d)
      if (!(a[d] > 0.0) || !std::isfinite(a[d]))
        return fail(ctx, SCFFT_ERR_ARG, "anisotropy weights must be finite and > 0");
  }
  const bool iso = !a || (a[0] == 1.0 && a[1] == 1.0 && a[2] == 1.0);
  for (int d = 0; d < 3; ++d) ctx->aniso_w[d] = iso ? 1.0 : a[d];
  ctx->has_aniso = !iso;
  return SCFFT_OK;
}

scfft_status scfft_set_rhs_opts(scfft_ctx* ctx, const scfft_rhs_opts* o) {
  if (!ctx || !o) return SCFFT_ERR_ARG;
  if (ctx->graph_busy) return fail(ctx, SCFFT_ERR_STATE, "a graph integration is enqueued");
  ++ctx->epoch;
  drop_cont(ctx);
  if (!(o->delta_it > 0.0) || o->min_iter < 0 || o->max_iter < 1 || o->fixed_iter < 0 ||
      !(o->sigma_scale > 0.0) || o->min_iter > o->max_iter || o->fuse_xy < 0 || o->fuse_xy > 2 ||
      o->x_alt < 0 || o->x_alt > 1 || o->y_alt < 0 || o->y_alt > 1 || o->z_alt < 0 || o->z_alt > 1)
    return fail(ctx, SCFFT_ERR_ARG, "invalid rhs options");
  const bool resigma = o->sigma_scale != ctx->opts.sigma_scale;
  ctx->opts = *o;
  if (resigma) {
    ctx->sigma = o->sigma_scale * 0.5 *
                 std::sqrt(ctx->h[0] * ctx->h[0] + ctx->h[1] * ctx->h[1] + ctx->h[2] * ctx->h[2]);
    if (ctx->ws) return ctx->prec == SCFFT_F64 ? upload_tables<double>(ctx) : upload_tables<float>(ctx);
  }
  return SCFFT_OK;
}

scfft_status scfft_get_rhs_opts(const scfft_ctx* ctx, scfft_rhs_opts* o) {
  if (!ctx || !o) return SCFFT_ERR_ARG;
  *o = ctx->opts;
  return SCFFT_OK;
}

scfft_status scfft_autotune(scfft_ctx* ctx, const void* h_dev, int32_t calls, int32_t* fuse_xy,
                            double* ms_per_call) {
  if (!ctx) return SCFFT_ERR_ARG;
  scfft_status st;
  if (!ready(ctx, true, &st)) return st;
  if (!ctx->has_drive) return fail(ctx, SCFFT_ERR_ARG, "no drive set");
  if (!h_dev || calls < 1) return fail(ctx, SCFFT_ERR_ARG, "invalid autotune arguments");
  CHECK_FIELD(ctx, h_dev);
  drop_cont(ctx);
  if (ctx->opts.fixed_iter <= 0)
    return fail(ctx, SCFFT_ERR_ARG, "autotune times a fixed iteration count (fixed_iter > 0)");
  int pick = 0;
  st = ctx->prec == SCFFT_F64 ? autotune_impl<double>(ctx, (const double*)h_dev, calls, &pick, ms_per_call)
                              : autotune_impl<float>(ctx, (const float*)h_dev, calls, &pick, ms_per_call);
  if (st == SCFFT_OK && fuse_xy) *fuse_xy = pick;
  return st;
}

scfft_status scfft_mask_betti(const scfft_ctx* ctx, int64_t betti[3]) {
  if (!ctx || !betti) return SCFFT_ERR_ARG;
  if (!ctx->has_mask) return SCFFT_ERR_GEOMETRY;
  for (int a = 0; a < 3; ++a) betti[a] = ctx->betti[a];
  return betti[1] > 0 ? SCFFT_WARN_TOPOLOGY : SCFFT_OK;
}

scfft_status scfft_reset_warm(scfft_ctx* ctx) {
  if (!ctx) return SCFFT_ERR_ARG;
  if (ctx->graph_busy) return fail(ctx, SCFFT_ERR_STATE, "a graph integration is enqueued");
  ctx->has_warm = false;
  drop_cont(ctx);
  return SCFFT_OK;
}

scfft_status scfft_init_state(scfft_ctx* ctx, double t0_s, void* h_dev) {
  if (!ctx || !h_dev) return SCFFT_ERR_ARG;
  CHECK_FIELD(ctx, h_dev);
  if (!ctx->has_drive) return fail(ctx, SCFFT_ERR_ARG, "no drive set");
  drop_cont(ctx);
  double he[3], hd[3];
  ctx->drive.eval(t0_s / ctx->u.t0, he, hd);
  hipError_t e = ctx->prec == SCFFT_F64
                     ? launch_fill_uniform<double>((double*)h_dev, ctx->nodes, he, ctx->stream)
                     : launch_fill_uniform<float>((float*)h_dev, ctx->nodes, he, ctx->stream);
  if (e != hipSuccess) return fail(ctx, SCFFT_ERR_DEVICE, "init_state: %s", hipGetErrorString(e));
  ctx->has_warm = false;
  return SCFFT_OK;
}

scfft_status scfft_rhs_eval(scfft_ctx* ctx, double t_s, const void* h_dev, void* hdot_dev,
                            scfft_rhs_stats* stats) {
  if (!ctx) return SCFFT_ERR_ARG;
  scfft_status st;
  if (!ready(ctx, true, &st)) return st;
  if (!h_dev || !hdot_dev) return fail(ctx, SCFFT_ERR_ARG, "NULL field pointer");
  if (h_dev == hdot_dev) return fail(ctx, SCFFT_ERR_ARG, "h and hdot must not alias");
  CHECK_FIELD(ctx, h_dev);
  CHECK_FIELD(ctx, hdot_dev);
  if (!ctx->has_drive) return fail(ctx, SCFFT_ERR_ARG, "no drive set");
  drop_cont(ctx);  // the warm start changes
  const double t = t_s / ctx->u.t0;
  return ctx->prec == SCFFT_F64
             ? rhs_impl<double>(ctx, t, (const double*)h_dev, (double*)hdot_dev, stats)
             : rhs_impl<float>(ctx, t, (const float*)h_dev, (float*)hdot_dev, stats);
}

scfft_status scfft_integrate(scfft_ctx* ctx, double t0_s, double t1_s, void* h_dev,
                             const scfft_ode_opts* o, scfft_observer obs, void* user,
                             scfft_ode_stats* stats) {
  if (!ctx) return SCFFT_ERR_ARG;
  scfft_status st;
  if (!ready(ctx, true, &st)) return st;
  if (!h_dev || !valid_ode_opts(o) || !(t1_s > t0_s))
    return fail(ctx, SCFFT_ERR_ARG, "invalid integrate arguments");
  CHECK_FIELD(ctx, h_dev);
  if (!ctx->has_drive) return fail(ctx, SCFFT_ERR_ARG, "no drive set");
  scfft_ode_stats local;
  scfft_ode_stats* s = stats ? stats : &local;
  std::memset(s, 0, sizeof *s);
  return ctx->prec == SCFFT_F64
             ? integrate_impl<double>(ctx, t0_s, t1_s, (double*)h_dev, o, obs, user, s)
             : integrate_impl<float>(ctx, t0_s, t1_s, (float*)h_dev, o, obs, user, s);
}

scfft_status scfft_rhs_vjp(scfft_ctx* ctx, const void* h_dev, int32_t warm_used,
                           const void* lam_dev, const void* mu_dev, void* hbar_dev, void* wbar_dev,
                           void* kappa_bar_dev, double* n_bar, double hedot_bar[3]) {
  if (!ctx) return SCFFT_ERR_ARG;
  scfft_status st;
  if (!ready(ctx, true, &st)) return st;
  if (!h_dev || !lam_dev || !hbar_dev) return fail(ctx, SCFFT_ERR_ARG, "NULL field pointer");
  if (hbar_dev == h_dev || hbar_dev == lam_dev || hbar_dev == mu_dev ||
      (wbar_dev && (wbar_dev == h_dev || wbar_dev == hbar_dev)))
    return fail(ctx, SCFFT_ERR_ARG, "outputs must not alias inputs");
  CHECK_FIELD(ctx, h_dev);
  CHECK_FIELD(ctx, lam_dev);
  CHECK_FIELD(ctx, mu_dev);
  CHECK_FIELD(ctx, hbar_dev);
  CHECK_FIELD(ctx, wbar_dev);
  if (ctx->opts.fixed_iter <= 0)
    return fail(ctx, SCFFT_ERR_ARG, "reverse mode needs a fixed iteration count (fixed_iter > 0)");
  drop_cont(ctx);
  double* sc = wsp<double>(ctx, ctx->off_adjs);
  HIPCHK(ctx, launch_zero_doubles(sc, 4, ctx->stream));
  st = ctx->prec == SCFFT_F64
           ? rhs_vjp_impl<double>(ctx, (const double*)h_dev, nullptr, 0.0, warm_used != 0,
                                  (const double*)lam_dev, (const double*)mu_dev, (double*)hbar_dev,
                                  (double*)wbar_dev, (double*)kappa_bar_dev, sc, 1.0)
           : rhs_vjp_impl<float>(ctx, (const float*)h_dev, nullptr, 0.0, warm_used != 0,
                                 (const float*)lam_dev, (const float*)mu_dev, (float*)hbar_dev,
                                 (float*)wbar_dev, (float*)kappa_bar_dev, sc, 1.0);
  if (st < 0) return st;
  double r[4];
  HIPCHK(ctx, hipMemcpyAsync(r, sc, sizeof r, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (n_bar) *n_bar = r[0];
  if (hedot_bar)
    for (int d = 0; d < 3; ++d) hedot_bar[d] = r[1 + d];
  return SCFFT_OK;
}

scfft_status scfft_adjoint_workspace_size(const scfft_ctx* ctx, int32_t steps,
                                          int32_t checkpoint_every, size_t* bytes) {
  if (!ctx || !bytes || steps <= 0 || checkpoint_every <= 0) return SCFFT_ERR_ARG;
  *bytes = adj_layout(ctx, steps, std::min(checkpoint_every, steps)).total;
  return SCFFT_OK;
}

scfft_status scfft_integrate_adjoint(scfft_ctx* ctx, double t0_s, double t1_s, int32_t steps,
                                     int32_t checkpoint_every, void* adj_ws, size_t adj_bytes,
                                     const void* h0_dev, const void* hT_bar_dev, void* hT_dev,
                                     void* h0_bar_dev, void* kappa_bar_dev, double* n_bar,
                                     double p_bar[3]) {
  if (!ctx) return SCFFT_ERR_ARG;
  scfft_status st;
  if (!ready(ctx, true, &st)) return st;
  if (!ctx->has_drive) return fail(ctx, SCFFT_ERR_ARG, "no drive set");
  if (steps <= 0 || checkpoint_every <= 0 || !(t1_s > t0_s))
    return fail(ctx, SCFFT_ERR_ARG, "invalid steps, checkpoint interval or time span");
  if (!h0_dev || !hT_bar_dev || !h0_bar_dev) return fail(ctx, SCFFT_ERR_ARG, "NULL field pointer");
  if (h0_bar_dev == h0_dev || h0_bar_dev == hT_bar_dev || (hT_dev && (hT_dev == h0_dev || hT_dev == h0_bar_dev)))
    return fail(ctx, SCFFT_ERR_ARG, "outputs must not alias inputs");
  CHECK_FIELD(ctx, h0_dev);
  CHECK_FIELD(ctx, hT_bar_dev);
  CHECK_FIELD(ctx, hT_dev);
  CHECK_FIELD(ctx, h0_bar_dev);
  if (ctx->opts.fixed_iter <= 0)
    return fail(ctx, SCFFT_ERR_ARG, "reverse mode needs a fixed iteration count (fixed_iter > 0)");
  drop_cont(ctx);
  if (p_bar && ctx->drive.kind == SCFFT_DRIVE_PWL)
    return fail(ctx, SCFFT_ERR_ARG, "p_bar needs a drive of the form p f(t) (ramp-hold or sine)");
  const int every = std::min<int>(checkpoint_every, steps);
  const AdjLayout L = adj_layout(ctx, steps, every);
  if (!adj_ws || adj_bytes < L.total || (reinterpret_cast<uintptr_t>(adj_ws) & 255))
    return fail(ctx, SCFFT_ERR_WORKSPACE, "adjoint workspace: %zu bytes at a 256-byte boundary needed",
                L.total);
  const double t0 = t0_s / ctx->u.t0, t1 = t1_s / ctx->u.t0;
  return ctx->prec == SCFFT_F64
             ? integrate_adjoint_impl<double>(ctx, t0, t1, steps, every, (char*)adj_ws, (double*)hT_dev,
                                              (const double*)h0_dev, (const double*)hT_bar_dev,
                                              (double*)h0_bar_dev, (double*)kappa_bar_dev, n_bar, p_bar)
             : integrate_adjoint_impl<float>(ctx, t0, t1, steps, every, (char*)adj_ws, (float*)hT_dev,
                                             (const float*)h0_dev, (const float*)hT_bar_dev,
                                             (float*)h0_bar_dev, (float*)kappa_bar_dev, n_bar, p_bar);
}

scfft_status scfft_graph_workspace_size(const scfft_ctx* ctx, int32_t steps, size_t* bytes) {
  if (!ctx || !bytes || steps <= 0) return SCFFT_ERR_ARG;
  *bytes = graph_layout(steps).total;
  return SCFFT_OK;
}

scfft_status scfft_integrate_graph(scfft_ctx* ctx, double t0_s, double t1_s, int32_t steps,
                                   void* graph_ws, size_t graph_bytes, void* h_dev) {
  if (!ctx) return SCFFT_ERR_ARG;
  scfft_status st;
  if (!ready(ctx, true, &st)) return st;
  if (!ctx->has_drive) return fail(ctx, SCFFT_ERR_ARG, "no drive set");
  if (!h_dev || steps <= 0 || !(t1_s > t0_s)) return fail(ctx, SCFFT_ERR_ARG, "invalid integrate arguments");
  CHECK_FIELD(ctx, h_dev);
  if (ctx->opts.fixed_iter <= 0)
    return fail(ctx, SCFFT_ERR_ARG, "graph replay needs a fixed iteration count (fixed_iter > 0)");
  drop_cont(ctx);
  const size_t need = graph_layout(steps).total;
  if (!graph_ws || graph_bytes < need || (reinterpret_cast<uintptr_t>(graph_ws) & 255))
    return fail(ctx, SCFFT_ERR_WORKSPACE, "graph workspace: %zu bytes at a 256-byte boundary needed", need);
  const double t0 = t0_s / ctx->u.t0, t1 = t1_s / ctx->u.t0;
  return ctx->prec == SCFFT_F64
             ? graph_begin_impl<double>(ctx, t0, t1, steps, (double*)h_dev, (char*)graph_ws)
             : graph_begin_impl<float>(ctx, t0, t1, steps, (float*)h_dev, (char*)graph_ws);
}

scfft_status scfft_integrate_wait(scfft_ctx* ctx, scfft_ode_stats* stats) {
  if (!ctx) return SCFFT_ERR_ARG;
  if (!ctx->graph_busy) return fail(ctx, SCFFT_ERR_STATE, "no graph integration is enqueued");
  return ctx->prec == SCFFT_F64 ? graph_wait_impl<double>(ctx, stats) : graph_wait_impl<float>(ctx, stats);
}

scfft_status scfft_graph_moments(scfft_ctx* ctx, int32_t omega_only, int32_t max_steps, double* m_Am2,
                                 int32_t* n_steps) {
  if (!ctx || !n_steps || max_steps < 0 || (max_steps > 0 && !m_Am2)) return SCFFT_ERR_ARG;
  if (ctx->graph_busy) return fail(ctx, SCFFT_ERR_STATE, "call scfft_integrate_wait first");
  if (ctx->graph_accepted < 0 || !ctx->graph_ws)
    return fail(ctx, SCFFT_ERR_STATE, "no graph integration has been waited for");
  const int n = std::min(max_steps, ctx->graph_accepted);
  *n_steps = ctx->graph_accepted;
  if (n == 0) return SCFFT_OK;
  const GraphLayout L = graph_layout(ctx->graph_steps);
  std::vector<double> h((size_t)n * 6);
  HIPCHK(ctx, hipMemcpyAsync(h.data(), ctx->graph_ws + L.off_mhist, h.size() * sizeof(double),
                             hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  const double dv = ctx->h[0] * ctx->h[1] * ctx->h[2];
  const double scale = ctx->u.jc * std::pow(ctx->u.l, 4.0);  // m' -> A m^2
  const int first = omega_only ? 3 : 0;
  for (int k = 0; k < n; ++k)
    for (int d = 0; d < 3; ++d) m_Am2[3 * (size_t)k + d] = 0.5 * h[6 * (size_t)k + first + d] * dv * scale;
  return SCFFT_OK;
}

scfft_status scfft_curl(scfft_ctx* ctx, const void* v_dev, void* out_dev) {
  if (!ctx) return SCFFT_ERR_ARG;
  scfft_status st;
  if (!ready(ctx, false, &st)) return st;
  if (!v_dev || !out_dev) return fail(ctx, SCFFT_ERR_ARG, "NULL field pointer");
  CHECK_FIELD(ctx, v_dev);
  CHECK_FIELD(ctx, out_dev);
  return ctx->prec == SCFFT_F64
             ? apply_operator<double>(ctx, (const double*)v_dev, (double*)out_dev, Z_CURL, 1.0)
             : apply_operator<float>(ctx, (const float*)v_dev, (float*)out_dev, Z_CURL, 1.0);
}

scfft_status scfft_phi(scfft_ctx* ctx, const void* v_dev, void* out_dev) {
  if (!ctx) return SCFFT_ERR_ARG;
  scfft_status st;
  if (!ready(ctx, false, &st)) return st;
  if (!v_dev || !out_dev) return fail(ctx, SCFFT_ERR_ARG, "NULL field pointer");
  CHECK_FIELD(ctx, v_dev);
  CHECK_FIELD(ctx, out_dev);
  const int sym = ctx->opts.smooth_phi ? Z_PHI_SMOOTH : Z_PHI;
  return ctx->prec == SCFFT_F64
             ? apply_operator<double>(ctx, (const double*)v_dev, (double*)out_dev, sym, 1.0)
             : apply_operator<float>(ctx, (const float*)v_dev, (float*)out_dev, sym, 1.0);
}

scfft_status scfft_curl_noalloc(scfft_ctx* ctx, const void* v_dev, void* out_dev) {
  if (!ctx) return SCFFT_ERR_ARG;
  if (ctx->graph_busy) return fail(ctx, SCFFT_ERR_STATE, "a graph integration is enqueued");
  if (!v_dev || !out_dev) return fail(ctx, SCFFT_ERR_ARG, "NULL field pointer");
  CHECK_FIELD(ctx, v_dev);
  CHECK_FIELD(ctx, out_dev);
  const size_t need = noalloc_bytes(ctx);
  if (need > kScratchBytes)
    return fail(ctx, SCFFT_ERR_WORKSPACE,
                "the allocation-free curl has %zu bytes of device scratch; this grid needs %zu",
                kScratchBytes, need);
  int dev = -1;
  HIPCHK(ctx, hipGetDevice(&dev));
  if (dev != ctx->device)
    return fail(ctx, SCFFT_ERR_DEVICE, "current device %d is not the context's (%d)", dev, ctx->device);
  char* base = nullptr;
  HIPCHK(ctx, scratch_on(dev, &base));
  return ctx->prec == SCFFT_F64
             ? curl_noalloc_impl<double>(ctx, base, (const double*)v_dev, (double*)out_dev)
             : curl_noalloc_impl<float>(ctx, base, (const float*)v_dev, (float*)out_dev);
}

scfft_status scfft_current(scfft_ctx* ctx, const void* h_dev, void* j_dev) {
  return scfft_curl(ctx, h_dev, j_dev);
}

scfft_status scfft_moment(scfft_ctx* ctx, const void* h_dev, int32_t omega_only, double m_Am2[3]) {
  if (!ctx) return SCFFT_ERR_ARG;
  scfft_status st;
  if (!ready(ctx, omega_only != 0, &st)) return st;
  if (!h_dev || !m_Am2) return fail(ctx, SCFFT_ERR_ARG, "NULL pointer");
  CHECK_FIELD(ctx, h_dev);
  return ctx->prec == SCFFT_F64 ? moment_impl<double>(ctx, (const double*)h_dev, omega_only, m_Am2)
                                : moment_impl<float>(ctx, (const float*)h_dev, omega_only, m_Am2);
}

scfft_status scfft_step_moment(scfft_ctx* ctx, int32_t omega_only, double m_Am2[3]) {
  if (!ctx || !m_Am2) return SCFFT_ERR_ARG;
  if (!ctx->ws) return fail(ctx, SCFFT_ERR_WORKSPACE, "no workspace attached");
  if (!ctx->obs_state ||
      (ctx->mom_sums_for != ctx->obs_state && ctx->mom_state != ctx->obs_state))
    return fail(ctx, SCFFT_ERR_STATE, "scfft_step_moment is valid inside an integrator observer only");
  const int first = omega_only ? 3 : 0;
  double r[3];
  if (ctx->mom_sums_for == ctx->obs_state) {  // read back with the step's error norm
    for (int d = 0; d < 3; ++d) r[d] = ctx->mom_sums[first + d];
  } else {
    const int xb = ctx->prec == SCFFT_F64 ? xpass_blocks<double>(make_plan<double>(ctx))
                                          : xpass_blocks<float>(make_plan<float>(ctx));
    const double* part = wsp<double>(ctx, ctx->off_mom);
    double* out = wsp<double>(ctx, ctx->off_mom) + 6 * ((size_t)ctx->n[1] * ctx->n[2]);
    HIPCHK(ctx, launch_sum_partials(part + first, xb, 6, 3, out, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(r, out, sizeof r, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  }
  const double dv = ctx->h[0] * ctx->h[1] * ctx->h[2];
  const double scale = ctx->u.jc * std::pow(ctx->u.l, 4.0);  // m' -> A m^2
  for (int d = 0; d < 3; ++d) m_Am2[d] = 0.5 * r[d] * dv * scale;
  return SCFFT_OK;
}

scfft_status scfft_region_mean_abs_b(scfft_ctx* ctx, const void* h_dev, const uint8_t* dev_region,
                                     double* b_T) {
  if (!ctx) return SCFFT_ERR_ARG;
  scfft_status st;
  if (!ready(ctx, false, &st)) return st;
  if (!h_dev || !dev_region || !b_T) return fail(ctx, SCFFT_ERR_ARG, "NULL pointer");
  CHECK_FIELD(ctx, h_dev);
  return ctx->prec == SCFFT_F64 ? region_impl<double>(ctx, (const double*)h_dev, dev_region, b_T)
                                : region_impl<float>(ctx, (const float*)h_dev, dev_region, b_T);
}

scfft_status scfft_stray_fraction(scfft_ctx* ctx, const void* h_dev, double* frac) {
  if (!ctx) return SCFFT_ERR_ARG;
  scfft_status st;
  if (!ready(ctx, true, &st)) return st;
  if (!h_dev || !frac) return fail(ctx, SCFFT_ERR_ARG, "NULL pointer");
  CHECK_FIELD(ctx, h_dev);
  return ctx->prec == SCFFT_F64 ? stray_impl<double>(ctx, (const double*)h_dev, frac)
                                : stray_impl<float>(ctx, (const float*)h_dev, frac);
}

scfft_status scfft_probe_b(scfft_ctx* ctx, const void* h_dev, const double* xyz_m, int32_t npts,
                           double* b_T) {
  if (!ctx) return SCFFT_ERR_ARG;
  scfft_status st;
  if (!ready(ctx, false, &st)) return st;
  if (!h_dev || npts < 0 || (npts > 0 && (!xyz_m || !b_T)))
    return fail(ctx, SCFFT_ERR_ARG, "invalid probe arguments");
  CHECK_FIELD(ctx, h_dev);
  for (int i = 0; i < 3 * npts; ++i)
    if (!std::isfinite(xyz_m[i])) return fail(ctx, SCFFT_ERR_ARG, "non-finite probe point");
  if (npts == 0) return SCFFT_OK;
  return ctx->prec == SCFFT_F64 ? probe_impl<double>(ctx, (const double*)h_dev, xyz_m, npts, b_T)
                                : probe_impl<float>(ctx, (const float*)h_dev, xyz_m, npts, b_T);
}

scfft_status scfft_get_state(scfft_ctx* ctx, void* blob, size_t* bytes) {
  if (!ctx || !bytes) return SCFFT_ERR_ARG;
  if (ctx->graph_busy) return fail(ctx, SCFFT_ERR_STATE, "a graph integration is enqueued");
  const size_t wb = ctx->has_warm ? 3 * ctx->nodes * ctx->wsize : 0;
  const bool k1 = ctx->cont.valid && ctx->cont.has_k1;
  const size_t kb = k1 ? 3 * ctx->nodes * ctx->wsize : 0;
  const size_t need = sizeof(StateHeader) + wb + kb;
  if (!blob) {
    *bytes = need;
    return SCFFT_OK;
  }
  if (*bytes < need) return fail(ctx, SCFFT_ERR_ARG, "state blob needs %zu bytes", need);
  StateHeader hd;
  std::memset(&hd, 0, sizeof hd);
  hd.magic = kStateMagic;
  hd.version = 2;
  hd.prec = ctx->prec;
  for (int a = 0; a < 3; ++a) hd.n[a] = ctx->n[a];
  hd.has_warm = ctx->has_warm ? 1 : 0;
  hd.opts = ctx->opts;
  hd.warm_bytes = wb;
  hd.iter_guess = ctx->iter_guess;
  hd.cont_valid = ctx->cont.valid ? 1 : 0;
  hd.cont_rejected = ctx->cont.rejected_last ? 1 : 0;
  hd.cont_has_k1 = k1 ? 1 : 0;
  hd.cont_t = ctx->cont.t;
  hd.cont_dt = ctx->cont.dt;
  hd.k1_bytes = kb;
  std::memcpy(blob, &hd, sizeof hd);
  if (wb)
    HIPCHK(ctx, hipMemcpyAsync((char*)blob + sizeof hd, ctx->ws + ctx->off_warm, wb,
                               hipMemcpyDeviceToHost, ctx->stream));
  if (kb)  // k1 sits in the K1 slot of the ODE buffers (one field each)
    HIPCHK(ctx, hipMemcpyAsync((char*)blob + sizeof hd + wb, ctx->ws + ctx->off_ode + (size_t)B_K1 * kb,
                               kb, hipMemcpyDeviceToHost, ctx->stream));
  if (wb || kb) HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  *bytes = need;
  return SCFFT_OK;
}

scfft_status scfft_set_state(scfft_ctx* ctx, const void* blob, size_t bytes) {
  if (!ctx || !blob) return SCFFT_ERR_ARG;
  if (ctx->graph_busy) return fail(ctx, SCFFT_ERR_STATE, "a graph integration is enqueued");
  scfft_status st;
  if (!ready(ctx, false, &st)) return st;
  StateHeader hd;
  if (bytes < sizeof hd) return fail(ctx, SCFFT_ERR_STATE, "state blob too short");
  std::memcpy(&hd, blob, sizeof hd);
  if (hd.magic != kStateMagic || hd.version != 2)
    return fail(ctx, SCFFT_ERR_STATE, "not an scfft state blob");
  if (hd.prec != ctx->prec || hd.n[0] != ctx->n[0] || hd.n[1] != ctx->n[1] || hd.n[2] != ctx->n[2])
    return fail(ctx, SCFFT_ERR_STATE, "state blob is for another grid or precision");
  const size_t fb = 3 * ctx->nodes * ctx->wsize;
  const size_t wb = hd.has_warm ? fb : 0;
  const size_t kb = hd.cont_has_k1 ? fb : 0;
  if (hd.warm_bytes != wb || hd.k1_bytes != kb || bytes < sizeof hd + wb + kb ||
      (hd.cont_has_k1 && !hd.cont_valid) || hd.iter_guess < 0 ||
      (hd.cont_valid && !(std::isfinite(hd.cont_t) && hd.cont_dt > 0.0 && std::isfinite(hd.cont_dt))))
    return fail(ctx, SCFFT_ERR_STATE, "state blob size mismatch");
  scfft_status s = scfft_set_rhs_opts(ctx, &hd.opts);  // drops the continuation
  if (s != SCFFT_OK) return s;
  if (wb)
    HIPCHK(ctx, hipMemcpyAsync(ctx->ws + ctx->off_warm, (const char*)blob + sizeof hd, wb,
                               hipMemcpyHostToDevice, ctx->stream));
  if (kb)
    HIPCHK(ctx, hipMemcpyAsync(ctx->ws + ctx->off_ode + (size_t)B_K1 * fb, (const char*)blob + sizeof hd + wb,
                               kb, hipMemcpyHostToDevice, ctx->stream));
  if (wb || kb) HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  ctx->has_warm = hd.has_warm != 0;
  ctx->iter_guess = hd.iter_guess;
  if (hd.cont_valid) {
    ctx->cont.valid = true;
    ctx->cont.t = hd.cont_t;
    ctx->cont.dt = hd.cont_dt;
    ctx->cont.rejected_last = hd.cont_rejected != 0;
    ctx->cont.has_k1 = hd.cont_has_k1 != 0;
  }
  return SCFFT_OK;
}

scfft_status scfft_profile(scfft_ctx* ctx, int32_t enable) {
  if (!ctx) return SCFFT_ERR_ARG;
  if (ctx->graph_busy) return fail(ctx, SCFFT_ERR_STATE, "a graph integration is enqueued");
  if (enable) {
    if (ctx->ev_pool.empty()) {
      const size_t pairs = 4096;
      ctx->ev_pool.resize(2 * pairs);
      ctx->ev_kind.resize(pairs);
      for (auto& e : ctx->ev_pool) HIPCHK(ctx, hipEventCreate(&e));
    }
    for (int k = 0; k < SCFFT_KERNEL_KINDS; ++k) {
      ctx->prof_launches[k] = 0;
      ctx->prof_ms[k] = 0.0;
      ctx->prof_bytes[k] = 0.0;
    }
    ctx->ev_used = 0;
    ctx->prof = true;
  } else {
    HIPCHK(ctx, prof_harvest(ctx));
    ctx->prof = false;
  }
  return SCFFT_OK;
}

scfft_status scfft_profile_read(scfft_ctx* ctx, int64_t launches[SCFFT_KERNEL_KINDS],
                                double total_ms[SCFFT_KERNEL_KINDS],
                                double total_bytes[SCFFT_KERNEL_KINDS]) {
  if (!ctx || !launches || !total_ms) return SCFFT_ERR_ARG;
  if (ctx->graph_busy) return fail(ctx, SCFFT_ERR_STATE, "a graph integration is enqueued");
  HIPCHK(ctx, prof_harvest(ctx));
  for (int k = 0; k < SCFFT_KERNEL_KINDS; ++k) {
    launches[k] = ctx->prof_launches[k];
    total_ms[k] = ctx->prof_ms[k];
    if (total_bytes) total_bytes[k] = ctx->prof_bytes[k];
  }
  return SCFFT_OK;
}

const char* scfft_status_string(scfft_status s) {
  switch (s) {
    case SCFFT_OK: return "ok";
    case SCFFT_WARN_NOT_CONVERGED: return "warning: exterior iteration did not converge";
    case SCFFT_WARN_CLAMPED: return "warning: power-law exponent clamped";
    case SCFFT_WARN_TOPOLOGY: return "warning: Omega is not contourwise simply connected";
    case SCFFT_ERR_ARG: return "invalid argument";
    case SCFFT_ERR_SHAPE: return "unsupported grid size";
    case SCFFT_ERR_DEVICE: return "device error";
    case SCFFT_ERR_WORKSPACE: return "workspace missing, too small or misaligned";
    case SCFFT_ERR_NAN: return "non-finite values";
    case SCFFT_ERR_STEP_UNDERFLOW: return "step size underflow";
    case SCFFT_ERR_GEOMETRY: return "geometry / mask missing";
    case SCFFT_ERR_STATE: return "state blob does not fit";
  }
  return "unknown status";
}

const char* scfft_last_error(const scfft_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

scfft_status scfft_batch_create(scfft_batch** out, scfft_ctx* const* members, int32_t count) {
  if (!out || !members || count < 1 || count > kMaxBatch) return SCFFT_ERR_ARG;
  *out = nullptr;
  scfft_ctx* c = members[0];
  if (!c) return SCFFT_ERR_ARG;
  for (int32_t b = 0; b < count; ++b) {
    scfft_ctx* m = members[b];
    if (!m) return fail(c, SCFFT_ERR_ARG, "member %d is NULL", b);
    for (int32_t q = 0; q < b; ++q)
      if (members[q] == m) return fail(c, SCFFT_ERR_ARG, "member %d appears twice", b);
    scfft_status st;
    if (!ready(m, true, &st)) return fail(c, st, "member %d: %s", b, m->err.c_str());
    if (!m->has_drive) return fail(c, SCFFT_ERR_ARG, "member %d has no drive", b);
    bool same = m->prec == c->prec && m->stream == c->stream && m->device == c->device;
    for (int a = 0; a < 3; ++a)
      same = same && m->n[a] == c->n[a] && std::fabs(m->L[a] - c->L[a]) <= 1e-12 * c->L[a];
    if (!same)
      return fail(c, SCFFT_ERR_SHAPE, "member %d differs in grid, dimensionless box, precision or stream", b);
    const scfft_rhs_opts &o = m->opts, &o0 = c->opts;
    if (o.fixed_iter <= 0 || o.fixed_iter != o0.fixed_iter || o.smooth_phi != o0.smooth_phi ||
        o.sigma_scale != o0.sigma_scale || o.fuse_xy != o0.fuse_xy || o.prune_box != o0.prune_box ||
        o.x_alt != o0.x_alt || o.y_alt != o0.y_alt || o.z_alt != o0.z_alt)
      return fail(c, SCFFT_ERR_ARG, "member %d: batches need equal options with fixed_iter > 0", b);
    if (m->field_hk_inv > 0.0 || m->has_aniso || m->has_kappa != c->has_kappa)
      return fail(c, SCFFT_ERR_ARG, "member %d: no field law or anisotropy, and jc maps on all or none", b);
  }
  // workspaces at a constant stride: instance b's buffers are instance 0's plus b strides
  size_t stride = 0;
  if (count > 1) {
    const uintptr_t w0 = (uintptr_t)c->ws, w1 = (uintptr_t)members[1]->ws;
    stride = w1 > w0 ? (size_t)(w1 - w0) : 0;
    if (stride < c->total || stride % kAlign)
      return fail(c, SCFFT_ERR_WORKSPACE, "member workspaces must follow each other at a constant stride");
    for (int32_t b = 2; b < count; ++b)
      if ((uintptr_t)members[b]->ws != w0 + (uintptr_t)b * stride)
        return fail(c, SCFFT_ERR_WORKSPACE, "member workspaces must follow each other at a constant stride");
  }
  scfft_batch* B = new scfft_batch();
  B->m.assign(members, members + count);
  B->stride = stride;
  // the box that holds Omega of every member (pruning stays exact)
  bool any = false;
  for (int a = 0; a < 3; ++a) {
    B->lo[a] = c->n[a];
    B->hi[a] = 0;
  }
  for (auto* m : B->m) {
    if (m->n_in == 0) continue;
    any = true;
    for (int a = 0; a < 3; ++a) {
      B->lo[a] = std::min(B->lo[a], m->box_lo[a]);
      B->hi[a] = std::max(B->hi[a], m->box_hi[a]);
    }
  }
  if (!any)
    for (int a = 0; a < 3; ++a) B->lo[a] = B->hi[a] = 0;
  hipError_t e = hipHostMalloc((void**)&B->pin, (size_t)kBatchRing * count * kBParDoubles * sizeof(double),
                               hipHostMallocDefault);
  for (int k = 0; k < kBatchRing && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&B->ev[k], hipEventDisableTiming);
  if (e != hipSuccess) {
    scfft_batch_destroy(B);
    return fail(c, SCFFT_ERR_DEVICE, "batch: %s", hipGetErrorString(e));
  }
  *out = B;
  return SCFFT_OK;
}

void scfft_batch_destroy(scfft_batch* B) {
  if (!B) return;
  if (!B->m.empty()) (void)hipStreamSynchronize(B->m[0]->stream);
  if (B->busy)
    for (auto* m : B->m) m->graph_busy = false;
  batch_drop_graphs(B);
  for (auto& ev : B->ev)
    if (ev) (void)hipEventDestroy(ev);
  if (B->pin) (void)hipHostFree(B->pin);
  delete B;
}

scfft_status scfft_batch_rhs_eval(scfft_batch* B, double t_s, const void* h_dev, void* hdot_dev,
                                  int64_t field_stride) {
  if (!B) return SCFFT_ERR_ARG;
  scfft_ctx* c = B->m[0];
  if (B->busy) return fail(c, SCFFT_ERR_STATE, "a batch graph integration is enqueued");
  if (!h_dev || !hdot_dev || h_dev == hdot_dev) return fail(c, SCFFT_ERR_ARG, "invalid field pointers");
  CHECK_FIELD(c, h_dev);
  CHECK_FIELD(c, hdot_dev);
  if (field_stride < (int64_t)(3 * c->nodes) || field_stride % 2)
    return fail(c, SCFFT_ERR_ARG, "field stride must be even and at least one field (3 Nx Ny Nz)");
  return c->prec == SCFFT_F64
             ? batch_rhs_impl<double>(B, t_s, (const double*)h_dev, (double*)hdot_dev, field_stride)
             : batch_rhs_impl<float>(B, t_s, (const float*)h_dev, (float*)hdot_dev, field_stride);
}

scfft_status scfft_batch_graph_workspace_size(const scfft_batch* B, int32_t steps, size_t* bytes) {
  if (!B || !bytes || steps <= 0) return SCFFT_ERR_ARG;
  *bytes = batch_graph_layout((int)B->m.size(), steps).total;
  return SCFFT_OK;
}

scfft_status scfft_batch_integrate_graph(scfft_batch* B, double t0_s, double t1_s, int32_t steps, void* graph_ws,
                                         size_t graph_bytes, void* h_dev, int64_t field_stride) {
  if (!B) return SCFFT_ERR_ARG;
  scfft_ctx* c = B->m[0];
  if (B->busy) return fail(c, SCFFT_ERR_STATE, "a batch graph integration is enqueued");
  scfft_status st;
  for (auto* m : B->m)
    if (!ready(m, true, &st)) return fail(c, st, "batch member: %s", m->err.c_str());
  if (!batch_warm(B, &st)) return st;
  if (!h_dev || steps <= 0 || !(t1_s > t0_s)) return fail(c, SCFFT_ERR_ARG, "invalid integrate arguments");
  CHECK_FIELD(c, h_dev);
  if (field_stride < (int64_t)(3 * c->nodes) || field_stride % 2)
    return fail(c, SCFFT_ERR_ARG, "field stride must be even and at least one field (3 Nx Ny Nz)");
  const size_t need = batch_graph_layout((int)B->m.size(), steps).total;
  if (!graph_ws || graph_bytes < need || (reinterpret_cast<uintptr_t>(graph_ws) & 255))
    return fail(c, SCFFT_ERR_WORKSPACE, "batch graph workspace: %zu bytes at a 256-byte boundary needed", need);
  for (auto* m : B->m) drop_cont(m);
  return c->prec == SCFFT_F64
             ? batch_graph_begin_impl<double>(B, t0_s, t1_s, steps, (char*)graph_ws, (double*)h_dev, field_stride)
             : batch_graph_begin_impl<float>(B, t0_s, t1_s, steps, (char*)graph_ws, (float*)h_dev, field_stride);
}

scfft_status scfft_batch_integrate_wait(scfft_batch* B, scfft_ode_stats* stats) {
  if (!B) return SCFFT_ERR_ARG;
  if (!B->busy) return fail(B->m[0], SCFFT_ERR_STATE, "no batch graph integration is enqueued");
  return B->m[0]->prec == SCFFT_F64 ? batch_graph_wait_impl<double>(B, stats)
                                    : batch_graph_wait_impl<float>(B, stats);
}

const char* scfft_batch_last_error(const scfft_batch* B) { return B ? B->m[0]->err.c_str() : ""; }

}  // extern "C"
