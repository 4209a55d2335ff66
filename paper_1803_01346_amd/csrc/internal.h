// Internal declarations shared by the host library and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "fft_core.h"

namespace scfft {

// Per-axis device tables (context precision T), built on the host in FP64:
//   tw[k]   = exp(-2 pi i k / N), k = 0..N-1
//   kodd[i] = pi m_i / L with m_i the signed DFT index, 0 at the Nyquist entry
//   kk[i]   = (pi m_i / L)^2 with the true Nyquist wavenumber
//   sm[i]   = exp(-sigma^2 (pi m_i / L)^2 / 2), the axis factor of S(k)
template <typename T>
struct AxisTab {
  const C2<T>* tw;
  const T* kodd;
  const T* kk;
  const T* sm;
};

// Spectrum and sizes seen by the pass kernels.
//   main[c][z][y][kx], kx = 0..nx/2-1   (x-transformed columns)
//   nyq [c][z][y]                       (the kx = nx/2 column)
// Index ranges that let passes skip work outside the bounding box of the
// superconductor (fields masked to Omega vanish outside it; rates that are
// masked afterwards are only needed inside it).  Half-open; full by default.
struct Ranges {
  int zlo, zhi;            // Y pass: planes processed;  Z pass: planes loaded (others 0)
  int ylo_in, yhi_in;      // Y pass: rows loaded (others 0)
  int ylo_out, yhi_out;    // Y pass: rows stored
  int zlo_out, zhi_out;    // Z pass: planes stored
  int xylo, xyhi, xzlo, xzhi;  // X pass: rows (y, z) processed
  int iylo, iyhi, izlo, izhi;  // X_HIN: rows whose inverse transform is needed
};

template <typename T>
struct Plan {
  int nx, ny, nz;
  C2<T>* main;
  AxisTab<T> ax, ay, az;
  Ranges r;
  const int* stop = nullptr;  // device flag: once nonzero, the passes of this plan return at once
  int xalt = 0;  // per-component X passes with the alternate element count per thread
  int yalt = 0;  // Y passes with the alternate element count per thread
  int zalt = 0;  // Z passes with the alternate element count per thread
  // batched launches: `batch` instances of the same grid, instance blockIdx.z;
  // instance b's spectrum starts zs_main elements after instance b-1's (the
  // axis tables are shared: equal grids and dimensionless boxes)
  int batch = 1;
  int64_t zs_main = 0;
  void full_ranges() {
    r = Ranges{0, nz, 0, ny, 0, ny, 0, nz, 0, ny, 0, nz, 0, ny, 0, nz};
  }
};

enum XOp : int {
  X_FWD = 0,      // real input -> spectrum
  X_LAW,          // spectrum -> j -> e (Eq. 1, rho_out outside) -> spectrum
  X_HIN,          // spectrum -> g = -curl e; hdot0 = chi g + (1-chi) warm -> out, spectrum
  X_MASK,         // spectrum -> chi * v -> spectrum
  X_UPDATE,       // spectrum -> phi; hdot = chi hdot + (1-chi)(hedot + phi) -> out, spectrum; |delta| sums
  X_UPDATE_LAST,  // X_UPDATE without the forward transform
  X_STORE,        // spectrum -> real output
  X_MOMENT,       // spectrum -> j; sums of r x j over all nodes (or chi nodes)
  // reverse mode of the right-hand side (fixed iteration count)
  X_ADJ_START,    // l = in + (1-chi) in2 -> out (running sum); (1-chi) l -> spectrum
  X_ADJ_ACC,      // spectrum -> l; out += l; (1-chi) l -> spectrum
  X_ADJ_LAST,     // spectrum -> l0; c = out; wbar = (1-chi) l0 -> warm_out;
                  // sums of (1-chi) c; gbar = chi c + (chi or 1) l0 -> spectrum
  X_ADJ_LAW,      // spectrum -> ebar; jbar = (de/dj)^T ebar at j = in -> spectrum;
                  // sums of ebar . e ln(|j|/kappa); kappa_bar += -n ebar . e / kappa
  X_NUM_OPS
};

enum ZSym : int { Z_CURL = 0, Z_PHI = 1, Z_PHI_SMOOTH = 2 };

// Fused xy-plane passes (one component, one z plane, plane held in LDS):
// Y inverse, X inverse, per-component pointwise step, X forward, Y forward.
enum XYOp : int {
  XY_FWD = 0,      // real input -> x, y forward
  XY_HIN,          // -curl e on Omega, warm start on Omega_out -> out (Omega), forward
  XY_MASK,         // chi * v, forward
  XY_UPDATE,       // exterior update of Eq. 5 with a fixed iteration count, forward
  XY_UPDATE_LAST,  // the same, storing hdot and the next warm start on Omega_out
  XY_STORE,        // real output
  XY_NUM_OPS
};
constexpr size_t kXYMaxLds = 160 * 1024;

template <typename T>
struct XArgs {
  const T* in;           // X_FWD: the input field is in + in2_coef * in2 (in2 may be null)
  const T* in2;
  T in2_coef;
  T* out;                // X_HIN, X_UPDATE*: hdot;  X_STORE: output field
  const T* warm;         // X_HIN: warm start (nullptr: Ohm-law start)
  const uint8_t* chi;    // mask [nz][ny][nx]
  const T* kappa;        // jc map or nullptr
  double* partials;      // X_UPDATE*: one double per block; X_MOMENT: 3 per block
  unsigned long long* clamps;
  T npow, rho_out, expmax;
  // X_LAW: field-dependent critical density kappa / (1 + |h| hk_inv)^kim_alpha,
  // h = in + in2_coef in2 read at Omega nodes; hk_inv = 0: independent of h
  T hk_inv, kim_alpha;
  // X_LAW: anisotropic law e = (|j|_A / kappa)^(n-1) A j / kappa, A = diag(aniso_w),
  // |j|_A^2 = sum_c aniso_w[c] j_c^2; aniso = 0: the isotropic law
  T aniso_w[3];
  int aniso;
  T hedot[3];
  int omega_only;        // X_MOMENT: 1 = chi nodes only
  int track;             // X_HIN, X_UPDATE*: 1 = keep every iterate in `out` and sum
                         // |delta| (adaptive stopping); 0 = fixed iteration count:
                         // only the nodes a later pass reads are touched
  T* warm_out;           // X_UPDATE_LAST with track = 0: also store hdot on Omega_out here
  double* mom_partials;  // X_LAW: if set, 6 doubles per block: sums of r x j over all
                         // nodes (3) and over Omega nodes (3), for the moment readout
  T* kappa_bar;          // X_ADJ_LAW: accumulated d/dkappa (scalar field) or nullptr
  T* j_out;              // X_LAW: if set, j = C_s h is also stored here (all nodes)
  // X_UPDATE*, XY_UPDATE*: if hedot_tab is set, the applied-field rate is
  // hedot_tab[9 * (*hedot_step) + 3 * hedot_stage + c] instead of hedot[c]
  // (graph replays of a step: one row of three stage rates per step)
  const double* hedot_tab;
  const int* hedot_step;
  int hedot_stage;
  int warm_used;         // X_ADJ_LAST: the forward call started from a warm start
  double pos0[3];        // coordinate of node 0 along each axis (moment)
  double step[3];        // node spacing (moment)
  // Batched launches (instance b = blockIdx.z): byte offsets of instance b's
  // pointers from instance 0's, b times the stride of their class:
  //   zs_ws   buffers inside the instances' workspaces (chi, kappa, warm,
  //           warm_out, partials, clamps, mom_partials, zpar)
  //   zs_in   in, in2;   zs_out   out, j_out;   zs_tab   hedot_tab
  // zpar (if set): per-instance scalars, [0] n, [1] rho_out, [2 + in2_sel]
  // the stage coefficient in2_coef (in2_sel >= 0)
  int64_t zs_ws, zs_in, zs_out, zs_tab;
  const double* zpar;
  int in2_sel;
};

// Instance b's pointer: p shifted by b * stride bytes (null stays null).
template <typename P>
__host__ __device__ __forceinline__ P* zshift(P* p, size_t bytes) {
  return p ? reinterpret_cast<P*>(reinterpret_cast<uintptr_t>(p) + bytes) : p;
}

// The arguments of instance blockIdx.z of a batched launch (unchanged for a
// single instance, where blockIdx.z = 0 and zpar is null).
template <typename T>
__device__ __forceinline__ XArgs<T> instance_args(const XArgs<T>& A0) {
  XArgs<T> A = A0;
  const size_t z = blockIdx.z;
  if (z) {
    const size_t w = z * (size_t)A.zs_ws, i = z * (size_t)A.zs_in, o = z * (size_t)A.zs_out;
    A.chi = zshift(A.chi, w);
    A.kappa = zshift(A.kappa, w);
    A.warm = zshift(A.warm, w);
    A.warm_out = zshift(A.warm_out, w);
    A.partials = zshift(A.partials, w);
    A.clamps = zshift(A.clamps, w);
    A.mom_partials = zshift(A.mom_partials, w);
    A.kappa_bar = zshift(A.kappa_bar, w);
    A.in = zshift(A.in, i);
    A.in2 = zshift(A.in2, i);
    A.out = zshift(A.out, o);
    A.j_out = zshift(A.j_out, o);
    A.hedot_tab = zshift(A.hedot_tab, z * (size_t)A.zs_tab);
  }
  if (A.zpar) {
    const double* q = zshift(A.zpar, z * (size_t)A.zs_ws);
    A.npow = (T)q[0];
    A.rho_out = (T)q[1];
    if (A.in2_sel >= 0) A.in2_coef = (T)q[2 + A.in2_sel];
  }
  return A;
}

// Optional start/stop events attached to a kernel's own dispatch (timing of
// the kernel body, as a kernel trace reports it); both null = plain launch.
struct KTime {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};

template <typename T>
int xpass_blocks(const Plan<T>& p);
template <typename T>
hipError_t launch_xpass(const Plan<T>& p, int op, const XArgs<T>& a, hipStream_t s, KTime t = {});
template <typename T>
hipError_t launch_ypass(const Plan<T>& p, bool inverse, hipStream_t s, KTime t = {});
template <typename T>
hipError_t launch_zpass(const Plan<T>& p, int sym, T coef, hipStream_t s, KTime t = {});
template <typename T>
bool xypass_supported(const Plan<T>& p);
template <typename T>
hipError_t launch_xypass(const Plan<T>& p, int op, const XArgs<T>& a, hipStream_t s, KTime t = {});

// ---- pointwise / reduction kernels (pointwise.hip) ----
hipError_t launch_sum_partials(const double* partials, int n, int stride, int ncomp, double* out,
                               hipStream_t s);
hipError_t launch_accum_partials(const double* partials, int n, int stride, int ncomp, double scale,
                                 double* out, hipStream_t s);
hipError_t launch_zero_doubles(double* p, int n, hipStream_t s);
// Device state of the stopping rule of iteration (5): flag (stop), iterations done, last mean
// |delta|.  iter_decide sums the per-block |delta| sums of one X_UPDATE pass and sets the flag
// when it >= min_iter and the mean over Omega_out nodes is below tol; it does nothing once
// the flag is set.
struct IterState {
  int stop;
  int iters;
  double last;
};
hipError_t launch_iter_reset(IterState* st, hipStream_t s);
// Device state of a graph-replayed fixed-step integration: stop flag (set at
// the first step whose error norm is not finite; every later kernel of the
// replays returns at once), accepted steps, first bad step (-1: none).
struct GraphState {
  int stop;
  int step;
  int bad;
  int pad;
};
hipError_t launch_graph_reset(GraphState* g, hipStream_t s);
// records err[0] as hist[step]; step += 1 if finite, else sets stop and bad
hipError_t launch_graph_step_end(const double* err, GraphState* g, double* hist, hipStream_t s);
// moment partials of the accepted state into its row of the history
hipError_t launch_graph_moment(const double* partials, int n, const GraphState* g, double* hist,
                               hipStream_t s);
hipError_t launch_iter_decide(const double* partials, int n, double n_out, double tol, int min_iter,
                              IterState* st, hipStream_t s);
template <typename T>
hipError_t launch_fill_uniform(T* h, size_t nodes, const double he[3], hipStream_t s);
// out = y + c1 k1 + c2 k2 + c3 k3 (terms with null k skipped)
template <typename T>
hipError_t launch_combo(T* out, const T* y, const T* k1, double c1, const T* k2, double c2,
                        const T* k3, double c3, size_t n, hipStream_t s, const int* stop = nullptr);
// per-block max of |dt (e1 k1 + e2 k2 + e3 k3 + e4 k4)| / max(|y|, |y1|, thr); NaN -> inf
template <typename T>
hipError_t launch_errnorm(const T* y, const T* y1, const T* k1, const T* k2, const T* k3,
                          const T* k4, double dt, double thr, size_t n, double* partials,
                          int nblocks, hipStream_t s, const int* stop = nullptr);
// per-block max of |a_i| / max(|y_i|, thr)
template <typename T>
hipError_t launch_ratio_max(const T* a, const T* y, double thr, size_t n, double* partials,
                            int nblocks, hipStream_t s);
hipError_t launch_max_partials(const double* partials, int n, double* out, hipStream_t s,
                               const int* stop = nullptr);
// per-block sums of |h| and count over region nodes
template <typename T>
hipError_t launch_region_abs(const T* h, const uint8_t* region, size_t nodes, double* partials,
                             int nblocks, hipStream_t s);
// per-block sums of |j|^2 over Omega_out and over Omega nodes
template <typename T>
hipError_t launch_mask_sq(const T* j, const uint8_t* chi, size_t nodes, double* partials,
                          int nblocks, hipStream_t s);
// trilinear probe of h at npts dimensionless points
template <typename T>
hipError_t launch_probe(const T* h, int nx, int ny, int nz, const double* pts, int npts,
                        double x0, double y0, double z0, double hx, double hy, double hz,
                        double* out, hipStream_t s);
template <typename T>
hipError_t launch_masked_copy(T* dst, const T* src, const uint8_t* chi, size_t nodes,
                              hipStream_t s);
// Batched integrator kernels (instance b = grid y): buffers of instance b lie
// b * zs bytes after instance 0's; par_b = par + b * zs bytes holds the
// instance's step coefficients (par_b[4..6]: stage weights times dt, [7]: dt)
template <typename T>
hipError_t launch_combo_batch(T* out, const T* y, const T* k1, const T* k2, const T* k3, const double* par,
                              size_t n, int count, int64_t zs, hipStream_t s, const int* stop);
template <typename T>
hipError_t launch_errnorm_batch(const T* y, const T* y1, const T* k1, const T* k2, const T* k3, const T* k4,
                                const double* par, double thr, size_t n, double* partials, int nblocks,
                                int count, int64_t zs, hipStream_t s, const int* stop);
hipError_t launch_max_partials_batch(const double* partials, int n, double* out, int count, int64_t zs,
                                     hipStream_t s, const int* stop);
// instance b (b < count) copies n values from src + b szs bytes to dst + b dzs bytes
template <typename T>
hipError_t launch_strided_copy(T* dst, int64_t dzs, const T* src, int64_t szs, size_t n, int count,
                               hipStream_t s);
hipError_t launch_batch_step_end(const double* err, int64_t zs, int count, int steps, GraphState* g,
                                 double* hist, hipStream_t s);
// the tables of one axis (AxisTab layout) computed on the device, in FP64
template <typename T>
hipError_t launch_axis_table(C2<T>* tw, T* kodd, T* kk, T* sm, int n, double L, double sigma,
                             hipStream_t s);
// per-block counts of values that are not finite and > 0 (jc map check)
template <typename T>
hipError_t launch_count_nonpositive(const T* v, size_t n, double* partials, int nblocks,
                                    hipStream_t s);

constexpr int kReduceBlocks = 1024;

}  // namespace scfft
