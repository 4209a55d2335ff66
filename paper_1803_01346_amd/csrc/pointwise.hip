// Streaming kernels outside the transform passes: the integrator's stage
// combinations and error norm, FP64 reductions, readouts.
//
// Reductions are two-stage and deterministic: a fixed grid writes one
// partial per block (fixed tree inside the block), and a single block sums
// or maximises the partials in a fixed order.  No floating-point atomics.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace scfft {

constexpr int kRB = 256;  // threads per block of these kernels

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kRB / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_max(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = kRB / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = fmax(sh[t], sh[t + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// out[c] = sum_b partials[b * stride + c], c < ncomp, one block.
__global__ __launch_bounds__(kRB) void sum_partials_kernel(const double* __restrict__ p, int n,
                                                           int stride, int ncomp,
                                                           double* __restrict__ out) {
  __shared__ double sh[kRB];
  for (int c = 0; c < ncomp; ++c) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kRB) acc += p[(size_t)i * stride + c];
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) out[c] = r;
  }
}

hipError_t launch_sum_partials(const double* partials, int n, int stride, int ncomp, double* out,
                               hipStream_t s) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(kRB), 0, s, partials, n, stride, ncomp,
                     out);
  return hipGetLastError();
}

// out[c] += scale * sum_b partials[b * stride + c], one block.
__global__ __launch_bounds__(kRB) void accum_partials_kernel(const double* __restrict__ p, int n,
                                                             int stride, int ncomp, double scale,
                                                             double* __restrict__ out) {
  __shared__ double sh[kRB];
  for (int c = 0; c < ncomp; ++c) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kRB) acc += p[(size_t)i * stride + c];
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) out[c] += scale * r;
  }
}

hipError_t launch_accum_partials(const double* partials, int n, int stride, int ncomp, double scale,
                                 double* out, hipStream_t s) {
  hipLaunchKernelGGL(accum_partials_kernel, dim3(1), dim3(kRB), 0, s, partials, n, stride, ncomp,
                     scale, out);
  return hipGetLastError();
}

__global__ void zero_doubles_kernel(double* __restrict__ p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0.0;
}

hipError_t launch_zero_doubles(double* p, int n, hipStream_t s) {
  hipLaunchKernelGGL(zero_doubles_kernel, dim3(1), dim3(64), 0, s, p, n);
  return hipGetLastError();
}

__global__ void iter_reset_kernel(IterState* st) {
  if (threadIdx.x == 0) {
    st->stop = 0;
    st->iters = 0;
    st->last = 0.0;
  }
}

__global__ void graph_reset_kernel(GraphState* g) {
  if (threadIdx.x == 0) {
    g->stop = 0;
    g->step = 0;
    g->bad = -1;
  }
}

hipError_t launch_graph_reset(GraphState* g, hipStream_t s) {
  hipLaunchKernelGGL(graph_reset_kernel, dim3(1), dim3(64), 0, s, g);
  return hipGetLastError();
}

__global__ void graph_step_end_kernel(const double* __restrict__ err, GraphState* g,
                                      double* __restrict__ hist) {
  if (threadIdx.x != 0 || g->stop) return;
  const double e = *err;
  hist[g->step] = e;
  if (!isfinite(e)) {
    g->stop = 1;
    g->bad = g->step;
  } else {
    g->step += 1;
  }
}

hipError_t launch_graph_step_end(const double* err, GraphState* g, double* hist, hipStream_t s) {
  hipLaunchKernelGGL(graph_step_end_kernel, dim3(1), dim3(64), 0, s, err, g, hist);
  return hipGetLastError();
}

// Graph replay: hist[6 * step + c] = sum_b partials[6 b + c] (the moment
// partials of the state just accepted, all nodes then Omega), summed in the
// order of sum_partials_kernel; nothing once the stop flag is set.
__global__ __launch_bounds__(kRB) void graph_moment_kernel(const double* __restrict__ p, int n,
                                                           const GraphState* g,
                                                           double* __restrict__ hist) {
  __shared__ double sh[kRB];
  if (g->stop) return;  // uniform across the block
  const int step = g->step;
  for (int c = 0; c < 6; ++c) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += kRB) acc += p[(size_t)i * 6 + c];
    const double r = block_sum(acc, sh);
    if (threadIdx.x == 0) hist[6 * (size_t)step + c] = r;
  }
}

hipError_t launch_graph_moment(const double* partials, int n, const GraphState* g, double* hist,
                               hipStream_t s) {
  hipLaunchKernelGGL(graph_moment_kernel, dim3(1), dim3(kRB), 0, s, partials, n, g, hist);
  return hipGetLastError();
}

hipError_t launch_iter_reset(IterState* st, hipStream_t s) {
  hipLaunchKernelGGL(iter_reset_kernel, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

__global__ __launch_bounds__(kRB) void iter_decide_kernel(const double* __restrict__ p, int n,
                                                          double n_out, double tol, int min_iter,
                                                          IterState* st) {
  __shared__ double sh[kRB];
  if (st->stop) return;  // uniform across the block
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kRB) acc += p[i];
  const double r = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    const int it = st->iters + 1;
    const double d = n_out > 0.0 ? r / n_out : 0.0;
    st->iters = it;
    st->last = d;
    if (it >= min_iter && d < tol) st->stop = 1;
  }
}

hipError_t launch_iter_decide(const double* partials, int n, double n_out, double tol, int min_iter,
                              IterState* st, hipStream_t s) {
  hipLaunchKernelGGL(iter_decide_kernel, dim3(1), dim3(kRB), 0, s, partials, n, n_out, tol, min_iter,
                     st);
  return hipGetLastError();
}

__global__ __launch_bounds__(kRB) void max_partials_kernel(const double* __restrict__ p, int n,
                                                           double* __restrict__ out,
                                                           const int* __restrict__ stop, int64_t zs) {
  __shared__ double sh[kRB];
  if (stop && *stop) return;  // uniform
  p = zshift(p, blockIdx.y * (size_t)zs);      // instance of a batched launch
  out = zshift(out, blockIdx.y * (size_t)zs);
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kRB) acc = fmax(acc, p[i]);
  const double r = block_max(acc, sh);
  if (threadIdx.x == 0) out[0] = r;
}

hipError_t launch_max_partials(const double* partials, int n, double* out, hipStream_t s,
                               const int* stop) {
  hipLaunchKernelGGL(max_partials_kernel, dim3(1), dim3(kRB), 0, s, partials, n, out, stop, (int64_t)0);
  return hipGetLastError();
}

hipError_t launch_max_partials_batch(const double* partials, int n, double* out, int count, int64_t zs,
                                     hipStream_t s, const int* stop) {
  hipLaunchKernelGGL(max_partials_kernel, dim3(1, count), dim3(kRB), 0, s, partials, n, out, stop, zs);
  return hipGetLastError();
}

// Batched graph replay: instance b's error norm (err + b zs bytes) into
// hist[b * steps + step]; a non-finite one stops every instance; else the
// shared step counter advances.
__global__ void batch_step_end_kernel(const double* __restrict__ err, int64_t zs, int count, int steps,
                                      GraphState* g, double* __restrict__ hist) {
  if (threadIdx.x != 0 || g->stop) return;
  bool bad = false;
  for (int b = 0; b < count; ++b) {
    const double e = *zshift(err, b * (size_t)zs);
    hist[(size_t)b * steps + g->step] = e;
    if (!isfinite(e)) bad = true;
  }
  if (bad) {
    g->stop = 1;
    g->bad = g->step;
  } else {
    g->step += 1;
  }
}

hipError_t launch_batch_step_end(const double* err, int64_t zs, int count, int steps, GraphState* g,
                                 double* hist, hipStream_t s) {
  hipLaunchKernelGGL(batch_step_end_kernel, dim3(1), dim3(64), 0, s, err, zs, count, steps, g, hist);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(kRB) void fill_uniform_kernel(T* __restrict__ h, size_t nodes, T a,
                                                           T b, T c) {
  for (size_t i = blockIdx.x * (size_t)kRB + threadIdx.x; i < nodes; i += (size_t)gridDim.x * kRB) {
    h[i] = a;
    h[nodes + i] = b;
    h[2 * nodes + i] = c;
  }
}

template <typename T>
hipError_t launch_fill_uniform(T* h, size_t nodes, const double he[3], hipStream_t s) {
  const int nb = (int)((nodes + kRB - 1) / kRB < 4096 ? (nodes + kRB - 1) / kRB : 4096);
  hipLaunchKernelGGL((fill_uniform_kernel<T>), dim3(nb), dim3(kRB), 0, s, h, nodes, (T)he[0],
                     (T)he[1], (T)he[2]);
  return hipGetLastError();
}

// out = y + c1 k1 + c2 k2 + c3 k3; coefficients in T (FP32 path: the stage
// combination is bulk arithmetic), terms with a null pointer are skipped.
// Batched (instance b = blockIdx.y): every buffer of instance b lies zs
// bytes after instance b-1's, and if par is set the coefficients are
// par_b[4], par_b[5], par_b[6] (par_b = par + b zs bytes).
template <typename T>
__global__ __launch_bounds__(kRB) void combo_kernel(T* __restrict__ out, const T* __restrict__ y,
                                                    const T* __restrict__ k1, T c1,
                                                    const T* __restrict__ k2, T c2,
                                                    const T* __restrict__ k3, T c3, size_t n,
                                                    const int* __restrict__ stop, int64_t zs,
                                                    const double* __restrict__ par) {
  if (stop && *stop) return;  // uniform
  if (blockIdx.y) {
    const size_t o = blockIdx.y * (size_t)zs;
    out = zshift(out, o);
    y = zshift(y, o);
    k1 = zshift(k1, o);
    k2 = zshift(k2, o);
    k3 = zshift(k3, o);
  }
  if (par) {
    const double* q = zshift(par, blockIdx.y * (size_t)zs);
    c1 = (T)q[4];
    c2 = (T)q[5];
    c3 = (T)q[6];
  }
  for (size_t i = blockIdx.x * (size_t)kRB + threadIdx.x; i < n; i += (size_t)gridDim.x * kRB) {
    T v = y ? y[i] : T(0);
    if (k1) v += c1 * k1[i];
    if (k2) v += c2 * k2[i];
    if (k3) v += c3 * k3[i];
    out[i] = v;
  }
}

template <typename T>
hipError_t launch_combo(T* out, const T* y, const T* k1, double c1, const T* k2, double c2,
                        const T* k3, double c3, size_t n, hipStream_t s, const int* stop) {
  const size_t want = (n + kRB - 1) / kRB;
  const int nb = (int)(want < 8192 ? want : 8192);
  hipLaunchKernelGGL((combo_kernel<T>), dim3(nb), dim3(kRB), 0, s, out, y, k1, (T)c1, k2, (T)c2,
                     k3, (T)c3, n, stop, (int64_t)0, (const double*)nullptr);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_combo_batch(T* out, const T* y, const T* k1, const T* k2, const T* k3, const double* par,
                              size_t n, int count, int64_t zs, hipStream_t s, const int* stop) {
  const size_t want = (n + kRB - 1) / kRB;
  const int nb = (int)(want < 2048 ? want : 2048);
  hipLaunchKernelGGL((combo_kernel<T>), dim3(nb, count), dim3(kRB), 0, s, out, y, k1, T(0), k2, T(0),
                     k3, T(0), n, stop, zs, par);
  return hipGetLastError();
}

// Error norm of the Bogacki-Shampine pair, FP64 regardless of T.
template <typename T>
__global__ __launch_bounds__(kRB) void errnorm_kernel(const T* __restrict__ y,
                                                      const T* __restrict__ y1,
                                                      const T* __restrict__ k1,
                                                      const T* __restrict__ k2,
                                                      const T* __restrict__ k3,
                                                      const T* __restrict__ k4, double dt,
                                                      double thr, size_t n,
                                                      double* __restrict__ partials,
                                                      const int* __restrict__ stop, int64_t zs,
                                                      const double* __restrict__ par) {
  __shared__ double sh[kRB];
  if (stop && *stop) return;  // uniform
  if (blockIdx.y) {  // instance of a batched launch (see combo_kernel)
    const size_t o = blockIdx.y * (size_t)zs;
    y = zshift(y, o);
    y1 = zshift(y1, o);
    k1 = zshift(k1, o);
    k2 = zshift(k2, o);
    k3 = zshift(k3, o);
    k4 = zshift(k4, o);
    partials = zshift(partials, o);
  }
  if (par) dt = zshift(par, blockIdx.y * (size_t)zs)[7];
  const double e1 = -5.0 / 72.0, e2 = 1.0 / 12.0, e3 = 1.0 / 9.0, e4 = -1.0 / 8.0;
  double acc = 0.0;
  for (size_t i = blockIdx.x * (size_t)kRB + threadIdx.x; i < n; i += (size_t)gridDim.x * kRB) {
    const double E = dt * (e1 * (double)k1[i] + e2 * (double)k2[i] + e3 * (double)k3[i] +
                           e4 * (double)k4[i]);
    const double sc = fmax(fmax(fabs((double)y[i]), fabs((double)y1[i])), thr);
    double r = fabs(E) / sc;
    if (!(r == r) || isinf(r)) r = INFINITY;  // NaN or inf forces rejection
    acc = fmax(acc, r);
  }
  const double r = block_max(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

template <typename T>
hipError_t launch_errnorm(const T* y, const T* y1, const T* k1, const T* k2, const T* k3,
                          const T* k4, double dt, double thr, size_t n, double* partials,
                          int nblocks, hipStream_t s, const int* stop) {
  hipLaunchKernelGGL((errnorm_kernel<T>), dim3(nblocks), dim3(kRB), 0, s, y, y1, k1, k2, k3, k4,
                     dt, thr, n, partials, stop, (int64_t)0, (const double*)nullptr);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_errnorm_batch(const T* y, const T* y1, const T* k1, const T* k2, const T* k3, const T* k4,
                                const double* par, double thr, size_t n, double* partials, int nblocks,
                                int count, int64_t zs, hipStream_t s, const int* stop) {
  hipLaunchKernelGGL((errnorm_kernel<T>), dim3(nblocks, count), dim3(kRB), 0, s, y, y1, k1, k2, k3, k4,
                     0.0, thr, n, partials, stop, zs, par);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(kRB) void ratio_max_kernel(const T* __restrict__ a,
                                                        const T* __restrict__ y, double thr,
                                                        size_t n, double* __restrict__ partials) {
  __shared__ double sh[kRB];
  double acc = 0.0;
  for (size_t i = blockIdx.x * (size_t)kRB + threadIdx.x; i < n; i += (size_t)gridDim.x * kRB) {
    double r = fabs((double)a[i]) / fmax(fabs((double)y[i]), thr);
    if (!(r == r)) r = INFINITY;
    acc = fmax(acc, r);
  }
  const double r = block_max(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

template <typename T>
hipError_t launch_ratio_max(const T* a, const T* y, double thr, size_t n, double* partials,
                            int nblocks, hipStream_t s) {
  hipLaunchKernelGGL((ratio_max_kernel<T>), dim3(nblocks), dim3(kRB), 0, s, a, y, thr, n, partials);
  return hipGetLastError();
}

// partials[2b] = sum |h| over region nodes, partials[2b+1] = count.
template <typename T>
__global__ __launch_bounds__(kRB) void region_abs_kernel(const T* __restrict__ h,
                                                         const uint8_t* __restrict__ region,
                                                         size_t nodes, double* __restrict__ partials) {
  __shared__ double sh[kRB];
  double acc = 0.0, cnt = 0.0;
  for (size_t i = blockIdx.x * (size_t)kRB + threadIdx.x; i < nodes; i += (size_t)gridDim.x * kRB) {
    if (region[i]) {
      const double a = h[i], b = h[nodes + i], c = h[2 * nodes + i];
      acc += sqrt(a * a + b * b + c * c);
      cnt += 1.0;
    }
  }
  const double s = block_sum(acc, sh);
  const double k = block_sum(cnt, sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = s;
    partials[2 * blockIdx.x + 1] = k;
  }
}

template <typename T>
hipError_t launch_region_abs(const T* h, const uint8_t* region, size_t nodes, double* partials,
                             int nblocks, hipStream_t s) {
  hipLaunchKernelGGL((region_abs_kernel<T>), dim3(nblocks), dim3(kRB), 0, s, h, region, nodes,
                     partials);
  return hipGetLastError();
}

// partials[2b] = sum of |j|^2 over Omega_out nodes, partials[2b+1] = over Omega.
template <typename T>
__global__ __launch_bounds__(kRB) void mask_sq_kernel(const T* __restrict__ j,
                                                      const uint8_t* __restrict__ chi,
                                                      size_t nodes, double* __restrict__ partials) {
  __shared__ double sh[kRB];
  double out = 0.0, in = 0.0;
  for (size_t i = blockIdx.x * (size_t)kRB + threadIdx.x; i < nodes; i += (size_t)gridDim.x * kRB) {
    const double a = j[i], b = j[nodes + i], c = j[2 * nodes + i];
    const double q = a * a + b * b + c * c;
    if (chi[i])
      in += q;
    else
      out += q;
  }
  const double so = block_sum(out, sh);
  const double si = block_sum(in, sh);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = so;
    partials[2 * blockIdx.x + 1] = si;
  }
}

template <typename T>
hipError_t launch_mask_sq(const T* j, const uint8_t* chi, size_t nodes, double* partials,
                          int nblocks, hipStream_t s) {
  hipLaunchKernelGGL((mask_sq_kernel<T>), dim3(nblocks), dim3(kRB), 0, s, j, chi, nodes, partials);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(kRB) void probe_kernel(const T* __restrict__ h, int nx, int ny, int nz,
                                                    const double* __restrict__ pts, int npts,
                                                    double x0, double y0, double z0, double hx,
                                                    double hy, double hz, double* __restrict__ out) {
  const int p = blockIdx.x * kRB + threadIdx.x;
  if (p >= npts) return;
  const double s[3] = {(pts[3 * p] - x0) / hx, (pts[3 * p + 1] - y0) / hy, (pts[3 * p + 2] - z0) / hz};
  const int nn[3] = {nx, ny, nz};
  int i0[3];
  double f[3];
  for (int a = 0; a < 3; ++a) {
    const double fl = floor(s[a]);
    f[a] = s[a] - fl;
    long long i = (long long)fl % nn[a];
    if (i < 0) i += nn[a];
    i0[a] = (int)i;
  }
  const size_t nodes = (size_t)nx * ny * nz;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const double w = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
        const int ix = (i0[0] + dx) % nx, iy = (i0[1] + dy) % ny, iz = (i0[2] + dz) % nz;
        const size_t idx = ((size_t)iz * ny + iy) * nx + ix;
        for (int c = 0; c < 3; ++c) acc[c] += w * (double)h[c * nodes + idx];
      }
  for (int c = 0; c < 3; ++c) out[3 * p + c] = acc[c];
}

template <typename T>
hipError_t launch_probe(const T* h, int nx, int ny, int nz, const double* pts, int npts, double x0,
                        double y0, double z0, double hx, double hy, double hz, double* out,
                        hipStream_t s) {
  hipLaunchKernelGGL((probe_kernel<T>), dim3((npts + kRB - 1) / kRB), dim3(kRB), 0, s, h, nx, ny,
                     nz, pts, npts, x0, y0, z0, hx, hy, hz, out);
  return hipGetLastError();
}

// dst = src on nodes outside Omega, 0 inside (warm start of iteration (5)).
template <typename T>
__global__ __launch_bounds__(kRB) void masked_copy_kernel(T* __restrict__ dst,
                                                          const T* __restrict__ src,
                                                          const uint8_t* __restrict__ chi,
                                                          size_t nodes) {
  for (size_t i = blockIdx.x * (size_t)kRB + threadIdx.x; i < nodes; i += (size_t)gridDim.x * kRB) {
    const bool in = chi[i] != 0;
    for (int c = 0; c < 3; ++c) dst[c * nodes + i] = in ? T(0) : src[c * nodes + i];
  }
}

template <typename T>
hipError_t launch_masked_copy(T* dst, const T* src, const uint8_t* chi, size_t nodes,
                              hipStream_t s) {
  const size_t want = (nodes + kRB - 1) / kRB;
  const int nb = (int)(want < 8192 ? want : 8192);
  hipLaunchKernelGGL((masked_copy_kernel<T>), dim3(nb), dim3(kRB), 0, s, dst, src, chi, nodes);
  return hipGetLastError();
}

// partials[b] = number of values in block b's share that are not finite and > 0
template <typename T>
__global__ __launch_bounds__(kRB) void count_nonpositive_kernel(const T* __restrict__ v, size_t n,
                                                                double* __restrict__ partials) {
  __shared__ double sh[kRB];
  double bad = 0.0;
  for (size_t i = blockIdx.x * (size_t)kRB + threadIdx.x; i < n; i += (size_t)gridDim.x * kRB) {
    const T x = v[i];
    if (!(x > T(0)) || !__builtin_isfinite(x)) bad += 1.0;  // NaN fails the first test
  }
  const double b = block_sum(bad, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = b;
}

template <typename T>
hipError_t launch_count_nonpositive(const T* v, size_t n, double* partials, int nblocks,
                                    hipStream_t s) {
  hipLaunchKernelGGL((count_nonpositive_kernel<T>), dim3(nblocks), dim3(kRB), 0, s, v, n, partials);
  return hipGetLastError();
}

// Batched set-up copies: instance b's n values of T go from src + b szs
// bytes to dst + b dzs bytes (instance b = blockIdx.y).
template <typename T>
__global__ __launch_bounds__(kRB) void strided_copy_kernel(T* __restrict__ dst, int64_t dzs,
                                                           const T* __restrict__ src, int64_t szs,
                                                           size_t n) {
  dst = zshift(dst, blockIdx.y * (size_t)dzs);
  src = zshift(src, blockIdx.y * (size_t)szs);
  for (size_t i = blockIdx.x * (size_t)kRB + threadIdx.x; i < n; i += (size_t)gridDim.x * kRB) dst[i] = src[i];
}

template <typename T>
hipError_t launch_strided_copy(T* dst, int64_t dzs, const T* src, int64_t szs, size_t n, int count,
                               hipStream_t s) {
  const size_t want = (n + kRB - 1) / kRB;
  const int nb = (int)(want < 2048 ? want : 2048);
  hipLaunchKernelGGL((strided_copy_kernel<T>), dim3(nb, count), dim3(kRB), 0, s, dst, dzs, src, szs, n);
  return hipGetLastError();
}
template hipError_t launch_strided_copy<double>(double*, int64_t, const double*, int64_t, size_t, int,
                                                hipStream_t);
template hipError_t launch_strided_copy<float>(float*, int64_t, const float*, int64_t, size_t, int,
                                               hipStream_t);

// The axis tables of one axis on the device (the layout of AxisTab):
// tw[i] = exp(-2 pi i / n), kodd[i] = pi m / L (0 at the Nyquist index),
// kk[i] = (pi m / L)^2, sm[i] = exp(-sigma^2 (pi m / L)^2 / 2), m the signed
// index of i.  Evaluated in FP64.
template <typename T>
__global__ __launch_bounds__(kRB) void axis_table_kernel(C2<T>* __restrict__ tw, T* __restrict__ kodd,
                                                         T* __restrict__ kk, T* __restrict__ sm, int n,
                                                         double L, double sigma) {
  const int i = blockIdx.x * kRB + threadIdx.x;
  if (i >= n) return;
  double sn, cs;
  sincospi(-2.0 * (double)i / (double)n, &sn, &cs);
  tw[i] = {(T)cs, (T)sn};
  const int m = 2 * i < n ? i : i - n;
  const double k = M_PI * (double)m / L;
  kodd[i] = (T)(2 * i == n ? 0.0 : k);
  kk[i] = (T)(k * k);
  sm[i] = (T)exp(-0.5 * sigma * sigma * k * k);
}

template <typename T>
hipError_t launch_axis_table(C2<T>* tw, T* kodd, T* kk, T* sm, int n, double L, double sigma,
                             hipStream_t s) {
  hipLaunchKernelGGL((axis_table_kernel<T>), dim3((n + kRB - 1) / kRB), dim3(kRB), 0, s, tw, kodd, kk, sm,
                     n, L, sigma);
  return hipGetLastError();
}

#define SCFFT_INST(T)                                                                          \
  template hipError_t launch_fill_uniform<T>(T*, size_t, const double[3], hipStream_t);        \
  template hipError_t launch_combo<T>(T*, const T*, const T*, double, const T*, double,        \
                                      const T*, double, size_t, hipStream_t, const int*);      \
  template hipError_t launch_errnorm<T>(const T*, const T*, const T*, const T*, const T*,      \
                                        const T*, double, double, size_t, double*, int,        \
                                        hipStream_t, const int*);                               \
  template hipError_t launch_region_abs<T>(const T*, const uint8_t*, size_t, double*, int,     \
                                           hipStream_t);                                        \
  template hipError_t launch_mask_sq<T>(const T*, const uint8_t*, size_t, double*, int,         \
                                        hipStream_t);                                           \
  template hipError_t launch_probe<T>(const T*, int, int, int, const double*, int, double,     \
                                      double, double, double, double, double, double*,         \
                                      hipStream_t);                                             \
  template hipError_t launch_masked_copy<T>(T*, const T*, const uint8_t*, size_t, hipStream_t); \
  template hipError_t launch_ratio_max<T>(const T*, const T*, double, size_t, double*, int,     \
                                          hipStream_t);                                         \
  template hipError_t launch_count_nonpositive<T>(const T*, size_t, double*, int, hipStream_t); \
  template hipError_t launch_axis_table<T>(C2<T>*, T*, T*, T*, int, double, double, hipStream_t); \
  template hipError_t launch_combo_batch<T>(T*, const T*, const T*, const T*, const T*, const double*, \
                                            size_t, int, int64_t, hipStream_t, const int*);     \
  template hipError_t launch_errnorm_batch<T>(const T*, const T*, const T*, const T*, const T*,  \
                                              const T*, const double*, double, size_t, double*,  \
                                              int, int, int64_t, hipStream_t, const int*);
SCFFT_INST(double)
SCFFT_INST(float)
#undef SCFFT_INST

}  // namespace scfft
