// Fused xy-plane pass: for one component and one z plane, the y inverse
// transform, the x inverse (complex-to-real), a per-component pointwise step,
// the x forward (real-to-complex) and the y forward transform, with the whole
// plane of the half spectrum held in LDS (Ny x (Nx/2 + 1) complex values; 133
// KB at 128 x 128 in FP64).  It replaces the three passes Y inverse, X, Y
// forward of the column/row schedule wherever the pointwise step needs one
// component at a time: the masks and the exterior update of iteration (5)
// with a fixed iteration count, the warm start, and the forward transform of
// a real field.  Global traffic is one read and one write of the plane.
//
// Plane layout in LDS: row y (fixed ky or y), entry k = kx (0..Nx/2), row
// stride Nx/2 + 1 (odd, so the y columns spread over the banks).  In HBM the
// kx = 0 column carries the Nyquist plane too (X[0] + i X[Nx/2] along x,
// half-complex along y; the layout note of the column passes); the plane
// unpacks it after loading and packs it before storing.  Columns are
// transformed by Ny/8 lanes each and rows by Nx/8 lanes each, always inside
// one wavefront, so every exchange needs only a wavefront barrier; block
// barriers separate the column and row phases.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"
#include "tuning.h"

namespace scfft {

// Threads per block (one block per plane), tuning.h.
template <typename T>
constexpr int xy_block() { return sizeof(T) == 8 ? tune::kXYBlockF64 : tune::kXYBlockF32; }

template <typename T, int STRIDE>
struct LdsLine {  // one row (STRIDE = 1) or one column (STRIDE = row stride) of the plane
  C2<T>* base;
  __device__ __forceinline__ void store(int idx, C2<T> v) { base[idx * STRIDE] = v; }
  __device__ __forceinline__ C2<T> load(int idx) const { return base[idx * STRIDE]; }
  __device__ __forceinline__ void sync() { wave_sync(); }
  __device__ __forceinline__ void after_load() { wave_sync(); }
};

template <typename T, int NX, int NY>
struct XYGeom {
  static constexpr int M = NX / 2;
  static constexpr int RS = M + 1;                      // plane row stride
  static constexpr int EY = elems_per_thread(NY, 8);
  static constexpr int TPTY = NY / EY;                  // lanes per column
  static constexpr int BLOCK = xy_block<T>();
  static constexpr int GY = BLOCK / TPTY;               // columns per round
  static constexpr int EX = elems_per_thread(M, 4);
  static constexpr int TPTX = M / EX;                   // lanes per row
  static constexpr int GX = BLOCK / TPTX;               // rows per round
  static constexpr int RX = (NY + GX - 1) / GX;         // row rounds
  static_assert(TPTY <= 64 && TPTX <= 64, "a line must fit one wavefront");
};

// y transforms of the M columns kx < Nx/2 of the plane, in place.
template <typename T, int NX, int NY, bool INV>
__device__ __forceinline__ void plane_columns(C2<T>* plane, const C2<T>* __restrict__ tw) {
  using G = XYGeom<T, NX, NY>;
  const int t = threadIdx.x;
  const int g = t / G::TPTY, j = t % G::TPTY;
  for (int col = g; col < G::M; col += G::GY) {
    LdsLine<T, G::RS> lds{plane + col};
    C2<T> v[G::EY];
#pragma unroll
    for (int m = 0; m < G::EY; ++m) v[m] = lds.load(j + m * G::TPTY);
    wave_sync();
    if constexpr (INV)
      fft_inverse<T, NY, G::EY>(v, j, lds, tw, 1);
    else
      fft_forward<T, NY, G::EY>(v, j, lds, tw, 1);
#pragma unroll
    for (int m = 0; m < G::EY; ++m) lds.store(j + m * G::TPTY, v[m]);
  }
}

// Complex-to-real x transform of one row (unnormalised): reals
// a[2m], a[2m+1] = x[2n], x[2n+1] with n = j + m TPTX.
template <typename T, int NX, int NY>
__device__ __forceinline__ void row_c2r(C2<T>* row, int j, const C2<T>* __restrict__ tw,
                                        T (&a)[2 * XYGeom<T, NX, NY>::EX]) {
  using G = XYGeom<T, NX, NY>;
  constexpr int M = G::M, E = G::EX, TPT = G::TPTX;
  C2<T> Z[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = j + m * TPT;
    const C2<T> X = row[k];
    const C2<T> pc = cconj(row[M - k]);                  // conj X[M-k]
    const C2<T> ev = X + pc;                             // X[k] + X[k+M]
    const C2<T> od = cmul(X - pc, cconj(tw[k]));         // (X[k] - X[k+M]) w^-k
    Z[m] = {ev.x - od.y, ev.y + od.x};                   // ev + i od
  }
  wave_sync();
  LdsLine<T, 1> lds{row};
  fft_inverse<T, M, E>(Z, j, lds, tw, 2);
#pragma unroll
  for (int m = 0; m < E; ++m) {
    a[2 * m] = Z[m].x;
    a[2 * m + 1] = Z[m].y;
  }
}

// Real-to-complex x transform of one row into row[0..M].
template <typename T, int NX, int NY>
__device__ __forceinline__ void row_r2c(C2<T>* row, int j, const C2<T>* __restrict__ tw,
                                        const T (&a)[2 * XYGeom<T, NX, NY>::EX]) {
  using G = XYGeom<T, NX, NY>;
  constexpr int M = G::M, E = G::EX, TPT = G::TPTX;
  C2<T> Z[E];
#pragma unroll
  for (int m = 0; m < E; ++m) Z[m] = {a[2 * m], a[2 * m + 1]};
  wave_sync();
  LdsLine<T, 1> lds{row};
  fft_forward<T, M, E>(Z, j, lds, tw, 2);
#pragma unroll
  for (int m = 0; m < E; ++m) row[j + m * TPT] = Z[m];
  wave_sync();
  C2<T> X[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int k = j + m * TPT;
    const C2<T> pc = cconj(row[(M - k) & (M - 1)]);      // conj Z[M-k], Z[M] = Z[0]
    const C2<T> s = Z[m] + pc, d = Z[m] - pc;
    const C2<T> ev = {T(0.5) * s.x, T(0.5) * s.y};       // E[k]
    const C2<T> od = {T(0.5) * d.y, T(-0.5) * d.x};      // O[k] = d / (2i)
    X[m] = ev + cmul(tw[k], od);
  }
  wave_sync();
  if (j == 0) X[0].y = Z[0].x - Z[0].y;                  // X[0] + i X[M] in the kx = 0 slot
#pragma unroll
  for (int m = 0; m < E; ++m) row[j + m * TPT] = X[m];
}

template <typename T, int NX, int NY, int OP>
__global__ __launch_bounds__(xy_block<T>()) void xyplane_kernel(Plan<T> P0, XArgs<T> A0) {
  using G = XYGeom<T, NX, NY>;
  constexpr int M = G::M, RS = G::RS, E = G::EX, TPT = G::TPTX;
  constexpr bool HAS_INV = OP != XY_FWD;
  constexpr bool HAS_FWD = OP == XY_FWD || OP == XY_HIN || OP == XY_MASK || OP == XY_UPDATE;
  constexpr bool NEED_CHI = OP == XY_HIN || OP == XY_MASK || OP == XY_UPDATE || OP == XY_UPDATE_LAST;
  constexpr bool NEED_AUX = OP == XY_FWD || OP == XY_HIN || OP == XY_UPDATE;
  __shared__ C2<T> plane[NY * RS];
  if (P0.stop && *P0.stop) return;  // uniform: a graph replay has stopped
  Plan<T> P = P0;
  P.main += blockIdx.z * P0.zs_main;  // instance of a batched launch
  const XArgs<T> A = instance_args(A0);

  const int nz = P.nz;
  const int nzr = P.r.zhi - P.r.zlo;                  // planes of this launch
  const int c = blockIdx.x / nzr;
  const int z = P.r.zlo + blockIdx.x % nzr;
  const int t = threadIdx.x;
  const int gx = t / TPT, j = t % TPT;
  const size_t csr = (size_t)nz * NY * NX;                    // component stride, real field
  const size_t rbase = (size_t)c * csr + (size_t)z * NY * NX;  // this plane, real field
  const size_t sbase = ((size_t)c * nz + z) * NY * M;          // this plane, spectrum
  // twiddle tables of both axes staged in LDS (fetched before the other loads)
  __shared__ C2<T> twl_x[NX];
  __shared__ C2<T> twl_y[NY];
  LdsTwiddles<T, NX, G::BLOCK> twdx;
  LdsTwiddles<T, NY, G::BLOCK> twdy;
  twdx.fetch(P.ax.tw);
  twdy.fetch(P.ay.tw);
  const C2<T>* twx = twl_x;
  // applied-field rate of this component, selected (a dynamic index into the
  // argument struct would copy it to scratch)
  T hdc = c == 0 ? A0.hedot[0] : (c == 1 ? A0.hedot[1] : A0.hedot[2]);
  if constexpr (OP == XY_UPDATE || OP == XY_UPDATE_LAST) {
    if (A.hedot_tab) hdc = (T)A.hedot_tab[9 * (size_t)(*A.hedot_step) + 3 * A.hedot_stage + c];
  }

  // per-node inputs of the rows this thread transforms, fetched first; the
  // mask of row round r is bit e of chm[r]
  static_assert(2 * E <= 32, "mask bits");
  // nodes x = 2n, 2n+1 of one complex element are adjacent: mask and real
  // fields are accessed two nodes at a time
  using T2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
  uint32_t chm[G::RX];
  T aux[NEED_AUX ? G::RX : 1][2 * E];
  const T* auxp = OP == XY_FWD ? A.in : (OP == XY_HIN ? A.warm : A.out);
#pragma unroll
  for (int r = 0; r < G::RX; ++r) {
    const int y = r * G::GX + gx;
    const bool ok = y < NY && (OP != XY_MASK || (y >= P.r.xylo && y < P.r.xyhi));
    uint32_t bits = 0;
    if constexpr (NEED_CHI) {
      const uint16_t* chp =
          reinterpret_cast<const uint16_t*>(A.chi + (size_t)z * NY * NX + (size_t)(ok ? y : 0) * NX);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const unsigned v = ok ? chp[j + m * TPT] : 0u;
        if (v & 0xffu) bits |= 1u << (2 * m);
        if (v >> 8) bits |= 2u << (2 * m);
      }
    }
    chm[r] = bits;
    if constexpr (NEED_AUX) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const size_t idx = rbase + (size_t)y * NX + 2 * (j + m * TPT);
        bool need[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const bool in = (bits >> (2 * m + h)) & 1u;
          bool nd = ok && auxp != nullptr;
          if constexpr (OP == XY_HIN) nd = nd && !in;     // warm start on Omega_out
          if constexpr (OP == XY_UPDATE) nd = nd && in;   // hdot_in on Omega
          need[h] = nd;
        }
        T2 v = {T(0), T(0)};
        if (need[0] || need[1]) {
          v = *reinterpret_cast<const T2*>(auxp + idx);
          if constexpr (OP == XY_FWD) {
            if (A.in2) {  // stage argument y + c k
              const T2 w = *reinterpret_cast<const T2*>(A.in2 + idx);
              v.x += A.in2_coef * w.x;
              v.y += A.in2_coef * w.y;
            }
          }
        }
        aux[r][2 * m] = need[0] ? v.x : T(0);
        aux[r][2 * m + 1] = need[1] ? v.y : T(0);
      }
    }
  }

  twdx.put(twl_x);
  twdy.put(twl_y);
  __syncthreads();  // line exchanges are wavefront-local: make the tables visible to the block

  // planes outside [izlo, izhi) need no inverse transform (their input counts as 0)
  const bool inv_plane = z >= P.r.izlo && z < P.r.izhi;
  if constexpr (HAS_INV) {
    if (inv_plane) {
      for (int i = t; i < NY * M; i += G::BLOCK) plane[(i / M) * RS + (i % M)] = P.main[sbase + i];
    } else {
      for (int i = t; i < NY * RS; i += G::BLOCK) plane[i] = C2<T>{T(0), T(0)};
    }
    __syncthreads();
    if (inv_plane) {  // uniform per block
      // kx = 0 column: P(ky) = A(ky) + i B(ky) from the half-complex layout
      for (int y = 1 + t; 2 * y < NY; y += G::BLOCK) {
        const C2<T> a = plane[y * RS], b = plane[(NY - y) * RS];
        plane[y * RS] = C2<T>{a.x - b.y, a.y + b.x};
        plane[(NY - y) * RS] = C2<T>{a.x + b.y, b.x - a.y};
      }
      __syncthreads();
      plane_columns<T, NX, NY, true>(plane, twl_y);
      __syncthreads();
      // X[0] + i X[M] of each row to the two real slots
      for (int y = t; y < NY; y += G::BLOCK) {
        const C2<T> pk = plane[y * RS];
        plane[y * RS] = C2<T>{pk.x, T(0)};
        plane[y * RS + M] = C2<T>{pk.y, T(0)};
      }
    }
    __syncthreads();
  }

#pragma unroll
  for (int r = 0; r < G::RX; ++r) {
    const int y = r * G::GX + gx;
    if (y < NY) {
      C2<T>* row = plane + y * RS;
      if constexpr (OP == XY_MASK) {
        if (y < P.r.xylo || y >= P.r.xyhi) {  // chi = 0 on rows outside the box: a zero row
#pragma unroll
          for (int m = 0; m < E; ++m) row[j + m * TPT] = C2<T>{T(0), T(0)};
          continue;
        }
      }
      T a[2 * E];
      if constexpr (HAS_INV) {
        row_c2r<T, NX, NY>(row, j, twx, a);
      } else {
#pragma unroll
        for (int e = 0; e < 2 * E; ++e) a[e] = aux[r][e];
      }
      uint32_t st_out = 0, st_warm = 0;  // bit e: store node e
#pragma unroll
      for (int e = 0; e < 2 * E; ++e) {
        const bool in = (chm[r] >> e) & 1u;
        if constexpr (OP == XY_HIN) {
          if (!in && A.warm) a[e] = aux[r][e];
          if (A.track || in) st_out |= 1u << e;
        } else if constexpr (OP == XY_MASK) {
          if (!in) a[e] = T(0);
        } else if constexpr (OP == XY_UPDATE) {
          a[e] = in ? aux[r][e] : hdc + a[e];
        } else if constexpr (OP == XY_UPDATE_LAST) {
          if (!in) {
            a[e] = hdc + a[e];
            st_out |= 1u << e;
            if (A.warm_out) st_warm |= 1u << e;
          }
        } else if constexpr (OP == XY_STORE) {
          st_out |= 1u << e;
        }
      }
      if constexpr (OP == XY_HIN || OP == XY_UPDATE_LAST || OP == XY_STORE) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
          const size_t idx = rbase + (size_t)y * NX + 2 * (j + m * TPT);
          const unsigned bo = (st_out >> (2 * m)) & 3u, bw = (st_warm >> (2 * m)) & 3u;
          const T v0 = a[2 * m], v1 = a[2 * m + 1];
          if (bo == 3u) {
            *reinterpret_cast<T2*>(A.out + idx) = T2{v0, v1};
          } else if (bo) {
            if (bo & 1u) A.out[idx] = v0;
            if (bo & 2u) A.out[idx + 1] = v1;
          }
          if (bw == 3u) {
            *reinterpret_cast<T2*>(A.warm_out + idx) = T2{v0, v1};
          } else if (bw) {
            if (bw & 1u) A.warm_out[idx] = v0;
            if (bw & 2u) A.warm_out[idx + 1] = v1;
          }
        }
      }
      if constexpr (HAS_FWD) row_r2c<T, NX, NY>(row, j, twx, a);
    }
  }

  if constexpr (HAS_FWD) {
    __syncthreads();
    plane_columns<T, NX, NY, false>(plane, twl_y);
    __syncthreads();
    // kx = 0 column to the half-complex layout: A(ky) and B(ky)
    for (int y = 1 + t; 2 * y < NY; y += G::BLOCK) {
      const C2<T> p = plane[y * RS], q = plane[(NY - y) * RS];
      plane[y * RS] = C2<T>{T(0.5) * (p.x + q.x), T(0.5) * (p.y - q.y)};
      plane[(NY - y) * RS] = C2<T>{T(0.5) * (p.y + q.y), T(0.5) * (q.x - p.x)};
    }
    __syncthreads();
    for (int i = t; i < NY * M; i += G::BLOCK) P.main[sbase + i] = plane[(i / M) * RS + (i % M)];
  }
}

// ---------------------------------------------------------------------------
template <typename T, int N>
static hipError_t xylaunch_n(const Plan<T>& p, int op, const XArgs<T>& a, hipStream_t s, KTime t) {
  const int nzr = p.r.zhi - p.r.zlo;
  if (nzr <= 0) return hipSuccess;
  const dim3 grid(3 * nzr, 1, p.batch), block(xy_block<T>());
#define SCFFT_XY_CASE(OPV)                                                                   \
  case OPV:                                                                                  \
    if (t.start)                                                                             \
      hipExtLaunchKernelGGL((xyplane_kernel<T, N, N, OPV>), grid, block, 0, s, t.start,      \
                            t.stop, 0, p, a);                                                \
    else                                                                                     \
      hipLaunchKernelGGL((xyplane_kernel<T, N, N, OPV>), grid, block, 0, s, p, a);           \
    break;
  switch (op) {
    SCFFT_XY_CASE(XY_FWD)
    SCFFT_XY_CASE(XY_HIN)
    SCFFT_XY_CASE(XY_MASK)
    SCFFT_XY_CASE(XY_UPDATE)
    SCFFT_XY_CASE(XY_UPDATE_LAST)
    SCFFT_XY_CASE(XY_STORE)
    default: return hipErrorInvalidValue;
  }
#undef SCFFT_XY_CASE
  return hipGetLastError();
}

template <typename T>
bool xypass_supported(const Plan<T>& p) {
  if (p.nx != p.ny) return false;
  const size_t lds = (size_t)p.ny * (p.nx / 2 + 1) * sizeof(C2<T>);
  return (p.nx == 16 || p.nx == 32 || p.nx == 64 || p.nx == 128) && lds <= kXYMaxLds;
}

template <typename T>
hipError_t launch_xypass(const Plan<T>& p, int op, const XArgs<T>& a, hipStream_t s, KTime t) {
  if (!xypass_supported(p)) return hipErrorInvalidValue;
  switch (p.nx) {
    case 16: return xylaunch_n<T, 16>(p, op, a, s, t);
    case 32: return xylaunch_n<T, 32>(p, op, a, s, t);
    case 64: return xylaunch_n<T, 64>(p, op, a, s, t);
    case 128: return xylaunch_n<T, 128>(p, op, a, s, t);
  }
  return hipErrorInvalidValue;
}

template bool xypass_supported<double>(const Plan<double>&);
template bool xypass_supported<float>(const Plan<float>&);
template hipError_t launch_xypass<double>(const Plan<double>&, int, const XArgs<double>&,
                                          hipStream_t, KTime);
template hipError_t launch_xypass<float>(const Plan<float>&, int, const XArgs<float>&, hipStream_t,
                                         KTime);

}  // namespace scfft
