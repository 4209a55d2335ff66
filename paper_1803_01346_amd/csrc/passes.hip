// The three kinds of full-field passes of one spectral operator application.
//
// A vector field v (3 components on an Nx x Ny x Nz grid) goes through
//   X pass   rows along x: real-to-complex transform of length Nx, done as a
//            complex transform of length Nx/2 plus a split step, fused with
//            all pointwise work of the method (power law, masks, exterior
//            update, reductions) between the inverse of one operator and
//            the forward transform of the next
//   Y pass   columns along y of the half spectrum (per component)
//   Z pass   columns along z, all three components at once: forward
//            transform, the operator's symbol (smoothed curl or Phi of
//            Eq. 7, both cross products with i k), inverse transform
// The spectrum of each component is stored as main[z][y][kx], kx < Nx/2,
// with the Nyquist plane (kx = Nx/2) packed into the kx = 0 column (see the
// note before the Y pass), so every row is a power of two long, column tiles
// stay aligned and the column passes have no leftover blocks.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"
#include "tuning.h"

namespace scfft {

constexpr int kBlock = 256;

// launch, with the events of t (if any) attached to the dispatch itself
template <typename F, typename... Args>
static void launch(F kernel, dim3 grid, dim3 block, hipStream_t s, KTime t, Args... args) {
  if (t.start)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, t.start, t.stop, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

// Elements per thread of each pass kind (tuning.h).
template <typename T, int NC = 3, int OP = -1>
constexpr int ex_max() {
  return NC == 1 ? (sizeof(T) == 8 ? tune::kEx1F64 : tune::kEx1F32)
                 : (sizeof(T) == 8 ? tune::kEx3F64 : tune::kEx3F32);
}
template <typename T>
constexpr int ey_max() { return sizeof(T) == 8 ? tune::kEyF64 : tune::kEyF32; }
template <typename T>
constexpr int ez_max() { return sizeof(T) == 8 ? tune::kEzF64 : tune::kEzF32; }

// Threads per block of a column pass: 256, doubled while the columns of one
// block span fewer than BYTES contiguous bytes of a row.
template <typename T, int N, int EMAX, int BYTES = tune::kColBytes>
constexpr int col_block() {
  const int tpt = N / elems_per_thread(N, EMAX);
  int b = kBlock;
  while ((b / tpt) * (int)sizeof(C2<T>) < BYTES && b < 1024) b *= 2;
  return b;
}

template <bool PP, typename T, int N, int COLS>
using ColLds = typename std::conditional<PP, LdsColsPP<T, N, COLS>, LdsCols<T, COLS>>::type;

// ---------------------------------------------------------------------------
// The kx = 0 column of the half spectrum carries two real x-spectra: the
// X pass stores X[0] + i X[Nx/2] there (both are real for a real field), so
// every row of the spectrum is a power of two long and no column is left
// over.  Along y the two are separated: after the forward y transform of
// that column, P(ky) = A(ky) + i B(ky) with A = F_y X[0] and B = F_y X[Nx/2]
// both Hermitian in ky, so the column is rewritten in a half-complex layout
//   slot ky   = A(ky)             1 <= ky < Ny/2
//   slot Ny-ky = B(ky)            1 <= ky < Ny/2
//   slot 0, Ny/2 = A + i B        (A and B real there)
// The Z pass transforms these columns like any other, using the Nyquist-plane
// wavevector (kx = Nx/2, Ny - ky) for the B columns and separating A and B
// along z in the two packed columns; the inverse y transform first rebuilds
// P(ky) from the half-complex layout.
// ---------------------------------------------------------------------------

// Y forward, kx = 0 column, slot y: P = P(y), Q = P(Ny - y).
template <typename T>
__device__ __forceinline__ C2<T> dc_split(C2<T> P, C2<T> Q, bool low) {
  if (low) return {T(0.5) * (P.x + Q.x), T(0.5) * (P.y - Q.y)};   // A(y) = (P + conj Q) / 2
  return {T(0.5) * (Q.y + P.y), T(0.5) * (P.x - Q.x)};             // B(Ny-y) = (Q - conj P) / 2i
}
// Y inverse, kx = 0 column, slot y: S = slot y, R = slot Ny - y.
template <typename T>
__device__ __forceinline__ C2<T> dc_join(C2<T> S, C2<T> R, bool low) {
  if (low) return {S.x - R.y, S.y + R.x};                          // A + i B, A = S, B = R
  return {R.x + S.y, S.x - R.y};                                   // conj(A) + i conj(B), A = R, B = S
}

// ---------------------------------------------------------------------------
// Y pass
// ---------------------------------------------------------------------------
// EV: elements-per-thread bound (0: ey_max; the alternate is a rhs option)
template <typename T, int NY, bool INV, int EV = 0>
__global__ __launch_bounds__((col_block<T, NY, EV ? EV : ey_max<T>()>())) void ypass_kernel(
    C2<T>* __restrict__ main, int M, int nz, Ranges R, const C2<T>* __restrict__ tw,
    const int* __restrict__ stop, int64_t zs) {
  if (stop && *stop) return;  // uniform: the iteration has stopped
  main += blockIdx.z * zs;    // instance of a batched launch
  constexpr int EM = EV ? EV : ey_max<T>();
  constexpr int E = elems_per_thread(NY, EM);
  constexpr int TPT = NY / E;
  constexpr int COLS = col_block<T, NY, EM>() / TPT;
  __shared__ C2<T> smem[(tune::kPingPongY ? 2 : 1) * NY * COLS];
  __shared__ C2<T> twl[NY];
  LdsTwiddles<T, NY, col_block<T, NY, EM>()> twd;
  twd.fetch(tw);
  const int tid = threadIdx.x;
  const int col = tid % COLS;
  const int j = tid / COLS;
  const int nzr = R.zhi - R.zlo;                       // planes processed
  const int q0 = (int)blockIdx.x * COLS;
  const int q = q0 + col;
  const bool valid = q < 3 * nzr * M;
  const int blk = q / M, kx = q % M;                   // blk = c * nzr + (z - zlo)
  const int c = blk / nzr, z = R.zlo + blk % nzr;
  C2<T>* p = main + ((size_t)c * nz + z) * NY * M + kx;
  const size_t es = (size_t)M;
  // blocks holding a kx = 0 column (uniform per block)
  const bool dc_block = (q0 % M == 0) || (q0 / M != (q0 + COLS - 1) / M);
  const bool dc = valid && kx == 0;
  C2<T> v[E];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int y = j + m * TPT;
    v[m] = (valid && y >= R.ylo_in && y < R.yhi_in) ? p[(size_t)y * es] : C2<T>{T(0), T(0)};
  }
  ColLds<tune::kPingPongY, T, NY, COLS> lds{smem, col};
  twd.put(twl);  // read from the transform's second pass on (block barriers between passes)
  if constexpr (INV) {
    if (dc_block) {  // rebuild P(ky) of the kx = 0 column from its half-complex layout
#pragma unroll
      for (int m = 0; m < E; ++m) smem[(j + m * TPT) * COLS + col] = v[m];
      __syncthreads();
      if (dc) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
          const int y = j + m * TPT;
          if (y != 0 && 2 * y != NY) v[m] = dc_join(v[m], smem[(NY - y) * COLS + col], 2 * y < NY);
        }
      }
      __syncthreads();
    }
    fft_inverse<T, NY, E>(v, j, lds, twl, 1);
  } else {
    fft_forward<T, NY, E>(v, j, lds, twl, 1);
    if (dc_block) {  // split the kx = 0 column into A and B (half-complex layout)
      __syncthreads();
#pragma unroll
      for (int m = 0; m < E; ++m) smem[(j + m * TPT) * COLS + col] = v[m];
      __syncthreads();
      if (dc) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
          const int y = j + m * TPT;
          if (y != 0 && 2 * y != NY) v[m] = dc_split(v[m], smem[(NY - y) * COLS + col], 2 * y < NY);
        }
      }
    }
  }
  if (valid) {
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int y = j + m * TPT;
      if (y >= R.ylo_out && y < R.yhi_out) p[(size_t)y * es] = v[m];
    }
  }
}

// ---------------------------------------------------------------------------
// Z pass: forward z transform of the three components, symbol, inverse.
// ---------------------------------------------------------------------------
// i f (k_odd x v) for one wavevector
template <typename T>
__device__ __forceinline__ void zsym_apply(C2<T>& a, C2<T>& b, C2<T>& d, T kxo, T kyo, T kzo, T f) {
  // k x v, then multiply by i f:  i (u + i w) f = (-w f, u f)
  const C2<T> cx = {kyo * d.x - kzo * b.x, kyo * d.y - kzo * b.y};
  const C2<T> cy = {kzo * a.x - kxo * d.x, kzo * a.y - kxo * d.y};
  const C2<T> cz = {kxo * b.x - kyo * a.x, kxo * b.y - kyo * a.y};
  a = {-cx.y * f, cx.x * f};
  b = {-cy.y * f, cy.x * f};
  d = {-cz.y * f, cz.x * f};
}

// Load through a buffer resource (base, size in bytes; gfx9 word 3): an offset
// at or past the size reads zero without touching memory.  Masked elements
// then need no branch, and a wave's loads stay in one straight line whose
// completions the compiler counts one by one, so a transform starts as soon
// as its own component has arrived.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
// An offset past every array read through one resource: each resource covers
// one component (edges up to 512: at most 512^3 FP64 values or 512^2 x 256
// complex FP64 values, 1 GiB), so sizes and offsets stay below 2^31.
constexpr unsigned kBufMiss = 0x80000000u;
template <typename T>
__device__ __forceinline__ T buffer_load_real(__amdgpu_buffer_rsrc_t r, unsigned off) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <typename T>
__device__ __forceinline__ C2<T> buffer_load(__amdgpu_buffer_rsrc_t r, unsigned off) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(C2<T>, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  else
    return __builtin_bit_cast(C2<T>, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

// FP64 default: at least 4 waves per SIMD, i.e. 4 blocks of 256 threads per
// CU, so the 1024 blocks of a 128 x 128 x 64 half spectrum run in one round on
// 256 CUs.  EV: elements-per-thread bound (0: ez_max; the alternate, a rhs
// option, takes the registers it needs).
template <typename T, int NZ, int EV>
constexpr int z_block() {
  return col_block<T, NZ, EV ? EV : ez_max<T>(), (sizeof(T) == 8 ? tune::kColBytesZF64 : tune::kColBytesZF32)>();
}
template <typename T, int NZ, int SYM, int EV = 0>
__global__ __launch_bounds__((z_block<T, NZ, EV>()), (sizeof(T) == 8 && EV == 0) ? 4 : 1) void zpass_kernel(
    C2<T>* __restrict__ main, int ny, int M, AxisTab<T> tx, AxisTab<T> ty, AxisTab<T> tz, T coef,
    Ranges R, const int* __restrict__ stop, int64_t zs) {
  if (stop && *stop) return;  // uniform: the iteration has stopped
  main += blockIdx.z * zs;    // instance of a batched launch
  constexpr int E = elems_per_thread(NZ, EV ? EV : ez_max<T>());
  constexpr int TPT = NZ / E;
  constexpr int COLS = z_block<T, NZ, EV>() / TPT;
  constexpr int BLOCK = z_block<T, NZ, EV>();
  // lane-swapped column transform where its layout fits (powers of two), else
  // Stockham passes; the former keeps its output in scrambled order
  using LC = LaneCol<T, NZ, E, COLS>;
  constexpr bool kLane = LC::ok && tune::kPingPongZ;
  __shared__ C2<T> smem[(tune::kPingPongZ ? 2 : 1) * NZ * COLS];
  __shared__ C2<T> twl[NZ];
  LdsTwiddles<T, NZ, BLOCK> twd;
  C2<T> twr[(NZ + BLOCK - 1) / BLOCK];
  if constexpr (kLane) {
    const __amdgpu_buffer_rsrc_t rt = buffer_of(tz.tw, NZ * sizeof(C2<T>));
#pragma unroll
    for (int k = 0; k < (NZ + BLOCK - 1) / BLOCK; ++k)
      twr[k] = buffer_load<T>(rt, (unsigned)((((int)threadIdx.x + k * BLOCK) & (NZ - 1)) * sizeof(C2<T>)));
  } else {
    twd.fetch(tz.tw);
  }
  const int tid = threadIdx.x;
  const int col = tid % COLS;
  const int j = tid / COLS;
  // blocks go to the 8 XCDs in turn; a column group of 64 bytes shares its
  // 128-byte lines with the next group: run the two on the same XCD
  int bx = (int)blockIdx.x;
  if (COLS * (int)sizeof(C2<T>) < 128 && gridDim.x % 8 == 0) bx = (bx % 8) * (int)(gridDim.x / 8) + bx / 8;
  const int q0 = bx * COLS;
  const int q = q0 + col;
  const bool valid = q < ny * M;
  C2<T>* p = main + q;
  const size_t es = (size_t)ny * M;
  const size_t cs = (size_t)NZ * ny * M;
  int kx = valid ? q % M : 0, ky = valid ? q / M : 0;
  // kx = 0 columns (see the layout note above): ky in (0, ny/2) hold A, the
  // kx = 0 plane; ky in (ny/2, ny) hold B of ky' = ny - ky, the Nyquist
  // plane; ky = 0 and ny/2 hold A + i B, separated along z below.
  const bool packed = valid && kx == 0 && (ky == 0 || 2 * ky == ny);
  if (kx == 0 && 2 * ky > ny) {
    kx = M;
    ky = ny - ky;
  }
  const int qa = (ny / 2) * M;                      // the second packed column
  const bool pk_block = q0 == 0 || (q0 <= qa && qa < q0 + COLS);  // uniform per block

  // The symbol's tables go to LDS with the twiddles: the z-axis arrays at
  // every kz and the x, y values of the block's columns, loaded before the
  // field loads, so the step between the transforms reads no global memory
  // (read there, they cost every block a round trip, and the blocks holding
  // the packed columns one per element).
  constexpr bool NEED_SM = SYM != Z_PHI, NEED_KK = SYM != Z_CURL;
  constexpr int NT1 = (NZ + BLOCK - 1) / BLOCK;
  __shared__ T zt[3 * NZ];     // kodd, sm, kk along z
  __shared__ T xyt[6 * COLS];  // per column: kodd x, kodd y, sm x, sm y, kk x, kk y
  T ztr[3][NT1];
  T xyr[6];
  {
    const T* za[3] = {tz.kodd, tz.sm, tz.kk};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if ((a == 1 && !NEED_SM) || (a == 2 && !NEED_KK)) continue;
      const __amdgpu_buffer_rsrc_t r = buffer_of(za[a], NZ * sizeof(T));
#pragma unroll
      for (int k = 0; k < NT1; ++k)
        ztr[a][k] = buffer_load_real<T>(r, (unsigned)((((int)threadIdx.x + k * BLOCK) % NZ) * sizeof(T)));
    }
    // the first COLS threads (j = 0) hold one column each
    const bool first = (int)threadIdx.x < COLS;
    const T* xa[6] = {tx.kodd, ty.kodd, tx.sm, ty.sm, tx.kk, ty.kk};
    const int xi[6] = {kx, ky, kx, ky, kx, ky};
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      if ((a / 2 == 1 && !NEED_SM) || (a / 2 == 2 && !NEED_KK)) continue;
      const __amdgpu_buffer_rsrc_t r = buffer_of(xa[a], (size_t)((a & 1) ? ny : 2 * M) * sizeof(T));
      xyr[a] = buffer_load_real<T>(r, first ? (unsigned)(xi[a] * sizeof(T)) : kBufMiss);
    }
  }
  // x values of the packed columns (kx = 0 and the Nyquist plane): uniform
  const T sx0 = NEED_SM ? tx.sm[0] : T(0), sxm = NEED_SM ? tx.sm[M] : T(0);
  const T qx0 = NEED_KK ? tx.kk[0] : T(0), qxm = NEED_KK ? tx.kk[M] : T(0);
  auto put_tables = [&]() {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if ((a == 1 && !NEED_SM) || (a == 2 && !NEED_KK)) continue;
#pragma unroll
      for (int k = 0; k < NT1; ++k) zt[a * NZ + (((int)threadIdx.x + k * BLOCK) % NZ)] = ztr[a][k];
    }
    if ((int)threadIdx.x < COLS) {
#pragma unroll
      for (int a = 0; a < 6; ++a) {
        if ((a / 2 == 1 && !NEED_SM) || (a / 2 == 2 && !NEED_KK)) continue;
        xyt[a * COLS + threadIdx.x] = xyr[a];
      }
    }
  };
  // multiplier of the symbol from its axis factors (sm, kk per axis)
  auto zfac = [&](T sxv, T qxv, T syv, T qyv, T szv, T qzv) -> T {
    if constexpr (SYM == Z_CURL) {
      return coef * sxv * syv * szv;
    } else {
      const T k2 = qxv + qyv + qzv;
      T f = k2 > T(0) ? coef / k2 : T(0);
      if constexpr (SYM == Z_PHI_SMOOTH) f = f * sxv * syv * szv;
      return f;
    }
  };
  // z of element m on load and store; kz of element m after the forward transform
  auto zpos = [&](int m) {
    if constexpr (kLane) return LC::pos_a(j, m);
    else return j + m * TPT;
  };
  auto kpos = [&](int m) {
    if constexpr (kLane) return LC::freq(j, m);
    else return j + m * TPT;
  };
  C2<T> v[3][E];
  ColLds<tune::kPingPongZ, T, NZ, COLS> lds{smem, col};
  if constexpr (kLane) {
    const size_t qc = valid ? (size_t)q : 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const __amdgpu_buffer_rsrc_t rc = buffer_of(main + c * cs, cs * sizeof(C2<T>));
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int z = zpos(m);
        const bool ok = valid && z >= R.zlo && z < R.zhi;
        v[c][m] = buffer_load<T>(rc, ok ? (unsigned)(((size_t)z * es + qc) * sizeof(C2<T>)) : kBufMiss);
      }
    }
#pragma unroll
    for (int k = 0; k < (NZ + BLOCK - 1) / BLOCK; ++k) twl[((int)threadIdx.x + k * BLOCK) & (NZ - 1)] = twr[k];
    put_tables();
    __syncthreads();  // the first step reads twiddles
#pragma unroll
    for (int c = 0; c < 3; ++c) LC::forward(v[c], j, col, smem + (c & 1) * NZ * COLS, twl);
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int z = j + m * TPT;
        v[c][m] = (valid && z >= R.zlo && z < R.zhi) ? p[c * cs + (size_t)z * es]
                                                     : C2<T>{T(0), T(0)};
      }
    twd.put(twl);  // read from the transform's second pass on (block barriers between passes)
    put_tables();
    __syncthreads();  // the tables, also where the transform has no exchange
#pragma unroll
    for (int c = 0; c < 3; ++c) fft_forward<T, NZ, E>(v[c], j, lds, twl, 1);
  }

  // Packed columns P = A + i B: with A = (P + conj P(-k)) / 2 on the kx = 0
  // plane and B = (P - conj P(-k)) / 2i on the Nyquist plane, and both planes
  // sharing k_odd = (0, ky, kz), the result A' + i B' of the symbols i f0 k x
  // and i fM k x equals i k x (a P + b conj P(-k)), a = (f0 + fM) / 2,
  // b = (f0 - fM) / 2.  conj P(-k) comes through LDS, one component at a time.
  if (pk_block) {
    T fa[E], fb[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int kz = kpos(m);
      const T sy = xyt[3 * COLS + col], qy = xyt[5 * COLS + col];
      const T sz = zt[NZ + kz], qz = zt[2 * NZ + kz];
      const T f0 = packed ? zfac(sx0, qx0, sy, qy, sz, qz) : T(0);
      const T fm = packed ? zfac(sxm, qxm, sy, qy, sz, qz) : T(0);
      fa[m] = T(0.5) * (f0 + fm);
      fb[m] = T(0.5) * (f0 - fm);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      __syncthreads();
#pragma unroll
      for (int m = 0; m < E; ++m) smem[kpos(m) * COLS + col] = v[c][m];
      __syncthreads();
      if (packed) {
#pragma unroll
        for (int m = 0; m < E; ++m) {
          const int kz = kpos(m);
          const C2<T> w = cconj(smem[(kz == 0 ? 0 : NZ - kz) * COLS + col]);
          v[c][m] = {fa[m] * v[c][m].x + fb[m] * w.x, fa[m] * v[c][m].y + fb[m] * w.y};
        }
      }
    }
    __syncthreads();
  }

  const T kxo = xyt[col], kyo = xyt[COLS + col];
  T fxy;  // the x, y part of the multiplier (packed columns: already applied)
  if constexpr (SYM == Z_CURL)
    fxy = coef * xyt[2 * COLS + col] * xyt[3 * COLS + col];
  else
    fxy = xyt[4 * COLS + col] + xyt[5 * COLS + col];
#pragma unroll
  for (int m = 0; m < E; ++m) {
    const int kz = kpos(m);
    T f;
    if constexpr (SYM == Z_CURL) {
      f = fxy * zt[NZ + kz];
    } else {
      const T k2 = fxy + zt[2 * NZ + kz];
      f = k2 > T(0) ? coef / k2 : T(0);
      if constexpr (SYM == Z_PHI_SMOOTH) f = f * xyt[2 * COLS + col] * xyt[3 * COLS + col] * zt[NZ + kz];
    }
    if (packed) f = T(1);
    zsym_apply(v[0][m], v[1][m], v[2][m], kxo, kyo, zt[kz], f);
  }
  // each component is stored as soon as its inverse is done, so its stores
  // overlap the inverse transforms of the next ones
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if constexpr (kLane)
      LC::inverse(v[c], j, col, smem + ((c + 1) & 1) * NZ * COLS, twl);
    else
      fft_inverse<T, NZ, E>(v[c], j, lds, twl, 1);
    if (valid) {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int z = zpos(m);
        if (z >= R.zlo_out && z < R.zhi_out) p[c * cs + (size_t)z * es] = v[c][m];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// X pass
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T dev_exp(T x);
template <>
__device__ __forceinline__ double dev_exp<double>(double x) { return exp(x); }
template <>
__device__ __forceinline__ float dev_exp<float>(float x) { return expf(x); }
template <typename T>
__device__ __forceinline__ T dev_log(T x);
template <>
__device__ __forceinline__ double dev_log<double>(double x) { return log(x); }
template <>
__device__ __forceinline__ float dev_log<float>(float x) { return logf(x); }
template <typename T>
__device__ __forceinline__ T dev_log1p(T x);
template <>
__device__ __forceinline__ double dev_log1p<double>(double x) { return log1p(x); }
template <>
__device__ __forceinline__ float dev_log1p<float>(float x) { return log1pf(x); }

// e = (|j|/kappa)^(n-1) j / kappa evaluated as j exp((n-1) (ln|j| - ln kappa) - ln kappa)
template <typename T>
__device__ __forceinline__ void power_law(T& a, T& b, T& c, T npow, T lnk, T expmax,
                                          unsigned& clamps) {
  const T s = a * a + b * b + c * c;
  if (s > T(0)) {
    T ex = (npow - T(1)) * (T(0.5) * dev_log<T>(s) - lnk) - lnk;
    if (ex > expmax) {
      ex = expmax;
      ++clamps;
    }
    const T f = dev_exp<T>(ex);
    a *= f;
    b *= f;
    c *= f;
  } else {
    a = T(0);
    b = T(0);
    c = T(0);
  }
}

// Anisotropic law (a user-chosen relation in place of Eq. 1, which the paper
// allows): the gradient in j of kappa/(n+1) (|j|_A/kappa)^(n+1), with
// |j|_A^2 = wx jx^2 + wy jy^2 + wz jz^2, that is e = (|j|_A/kappa)^(n-1) A j/kappa.
template <typename T>
__device__ __forceinline__ void power_law_aniso(T& a, T& b, T& c, T wx, T wy, T wz, T npow, T lnk,
                                                T expmax, unsigned& clamps) {
  const T s = wx * a * a + wy * b * b + wz * c * c;
  if (s > T(0)) {
    T ex = (npow - T(1)) * (T(0.5) * dev_log<T>(s) - lnk) - lnk;
    if (ex > expmax) {
      ex = expmax;
      ++clamps;
    }
    const T f = dev_exp<T>(ex);
    a *= wx * f;
    b *= wy * f;
    c *= wz * f;
  } else {
    a = T(0);
    b = T(0);
    c = T(0);
  }
}

// NC = 3: all three components per row (the power law, the moment, the
// exterior update with convergence sums); NC = 1: one component per block
// (blockIdx.y), for the steps that act on each component alone.
// EV: elements-per-thread bound of the row transform (0: the default of the
// op, ex_max); the schedule autotuner may pick the alternate one.
// The FP64 power-law pass on rows up to 128 is held to 4 waves per SIMD (128
// VGPRs): its 4096 waves at 128^3 then fit one round of the chip instead of
// 1.33 (at 146 VGPRs, 3 waves per SIMD); it spills 28 bytes per lane and is
// still faster (23.9 vs 25.8 us).  The same bound on X_HIN measured slower.
template <typename T, int NX, int OP, int NC, int EV = 0>
__global__ __launch_bounds__(kBlock, (sizeof(T) == 8 && OP == X_LAW && NC == 3 && NX <= 128) ? 4 : 1) void xpass_kernel(
    Plan<T> P0, XArgs<T> A0) {
  if (P0.stop && *P0.stop) return;  // uniform: the iteration has stopped
  Plan<T> P = P0;
  P.main += blockIdx.z * P0.zs_main;        // instance of a batched launch
  const XArgs<T> A = instance_args(A0);
  static_assert(NC == 3 || NC == 1, "components per block");
  static_assert(NC == 3 || (OP != X_LAW && OP != X_MOMENT && OP != X_ADJ_LAST && OP != X_ADJ_LAW),
                "needs all components");
  constexpr int M = NX / 2;
  constexpr int E = elems_per_thread(M, EV ? EV : ex_max<T, NC, OP>());
  constexpr int TPT = M / E;
  constexpr int ROWS = kBlock / TPT;
  static_assert(2 * E <= 32, "store masks hold one bit per node");
  constexpr bool HAS_INV = OP != X_FWD && OP != X_ADJ_START;
  constexpr bool HAS_FWD = OP == X_FWD || OP == X_LAW || OP == X_HIN || OP == X_MASK ||
                           OP == X_UPDATE || OP >= X_ADJ_START;
  constexpr bool REDUCE = OP == X_UPDATE || OP == X_UPDATE_LAST || OP == X_MOMENT ||
                          OP == X_ADJ_LAST || OP == X_ADJ_LAW;
  constexpr bool REDUCE3 = OP == X_MOMENT || OP == X_ADJ_LAST;  // 3 sums per block
  using L = LdsRows<T, M, E>;
  __shared__ C2<T> smem[ROWS * L::STRIDE];
  __shared__ double red[REDUCE ? 3 * kBlock : 1];

  const int tid = threadIdx.x;
  const int rl = tid / TPT;
  const int j = tid % TPT;
  const int nrows = P.ny * P.nz;
  const int nyb = P.r.xyhi - P.r.xylo;                 // rows processed: y, z in the range
  const int r = blockIdx.x * ROWS + rl;
  const bool valid = r < nyb * (P.r.xzhi - P.r.xzlo);
  const int ry = P.r.xylo + (valid ? r % nyb : 0);
  const int rz = P.r.xzlo + (valid ? r / nyb : 0);
  const int rr = rz * P.ny + ry;                       // global row index
  // rows whose inverse transform is needed (elsewhere the input counts as 0)
  const bool inv_row = valid && ry >= P.r.iylo && ry < P.r.iyhi && rz >= P.r.izlo && rz < P.r.izhi;
  const size_t csm = (size_t)nrows * M;        // component stride, main spectrum
  const size_t csr = (size_t)nrows * NX;       // component stride, real field
  __shared__ C2<T> twl[NX];
  constexpr int NTW = (NX + kBlock - 1) / kBlock;  // table entries per thread (duplicates allowed)
  C2<T> twr[NTW];
  {
    const __amdgpu_buffer_rsrc_t rt = buffer_of(P.ax.tw, NX * sizeof(C2<T>));
#pragma unroll
    for (int k = 0; k < NTW; ++k)
      twr[k] = buffer_load<T>(rt, (unsigned)((((int)threadIdx.x + k * kBlock) % NX) * sizeof(C2<T>)));
  }
  const C2<T>* tw = twl;                       // exp(-2 pi i k / NX), staged in LDS below
  const int c0 = NC == 3 ? 0 : (int)blockIdx.y;  // first component of this block
  L lds{smem, rl};

  T a[NC][2 * E];
  unsigned clamps = 0;
  T hdv[NC];  // applied-field rate of the exterior update
#pragma unroll
  for (int cc = 0; cc < NC; ++cc) hdv[cc] = A0.hedot[c0 + cc];  // kernel argument: indexed in place
  if constexpr (OP == X_UPDATE || OP == X_UPDATE_LAST) {
    if (A.hedot_tab) {
      const double* q = A.hedot_tab + 9 * (size_t)(*A.hedot_step) + 3 * A.hedot_stage;
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) hdv[cc] = (T)q[c0 + cc];
    }
  }
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0, acc4 = 0.0, acc5 = 0.0;
  const int y = rr % P.ny;
  const int z = rr / P.ny;
  const size_t rowbase = (size_t)rr * NX;

  // ---- all global loads first, so their latencies overlap.  Buffer loads
  // (an offset past the end reads zero) keep them free of branches, so the
  // compiler counts their completions one by one; the mask comes first, since
  // the loads of the real fields that depend on it come last ----
  constexpr bool NEED_CHI = OP != X_FWD && OP != X_STORE;
  constexpr bool NEED_AUX = OP == X_HIN || OP == X_UPDATE || OP == X_UPDATE_LAST || OP >= X_ADJ_START;
  // Nodes x = 2n, 2n+1 of one complex element n are adjacent: the mask and
  // the real fields are read (and stored) two nodes per access.  Measured
  // faster for every FP32 pass and for the FP64 updates; the FP64 input and
  // warm-start passes keep one node per access.
  constexpr bool PAIRED = sizeof(T) == 4 || !(OP == X_FWD || OP == X_HIN);
  uint8_t ch[2 * E];
  if constexpr (NEED_CHI) {
    const __amdgpu_buffer_rsrc_t rc = buffer_of(A.chi, (size_t)nrows * NX);
    if constexpr (!PAIRED) {
#pragma unroll
      for (int e = 0; e < 2 * E; ++e)
        ch[e] = __builtin_amdgcn_raw_buffer_load_b8(
            rc, valid ? (unsigned)(rowbase + 2 * (j + (e >> 1) * TPT) + (e & 1)) : kBufMiss, 0, 0);
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const unsigned v =
            __builtin_amdgcn_raw_buffer_load_b16(rc, valid ? (unsigned)(rowbase + 2 * (j + m * TPT)) : kBufMiss, 0, 0);
        ch[2 * m] = (uint8_t)(v & 0xffu);
        ch[2 * m + 1] = (uint8_t)(v >> 8);
      }
    }
  }
  C2<T> Xs[HAS_INV ? NC : 1][E];
  // the power law loads its third component's row after the first is transformed
  constexpr bool LAZY = NC == 3 && OP == X_LAW;
  auto load_row = [&](int cc) {
    const __amdgpu_buffer_rsrc_t rm = buffer_of(P.main + (c0 + cc) * csm, csm * sizeof(C2<T>));
#pragma unroll
    for (int m = 0; m < E; ++m)
      Xs[cc][m] = buffer_load<T>(rm, inv_row ? (unsigned)(((size_t)rr * M + j + m * TPT) * sizeof(C2<T>)) : kBufMiss);
  };
  if constexpr (HAS_INV) {
#pragma unroll
    for (int cc = 0; cc < (LAZY ? 2 : NC); ++cc) load_row(cc);
  }
  // the twiddle table goes to LDS before the loads that wait for the mask are
  // issued, so the transforms below do not wait for them
#pragma unroll
  for (int k = 0; k < NTW; ++k) twl[((int)threadIdx.x + k * kBlock) % NX] = twr[k];
  __syncthreads();  // row exchanges are wavefront-local: make the table visible to the block
  // X_FWD: the real input (all nodes); X_HIN: the warm start (Omega_out);
  // X_UPDATE*: hdot^i (all nodes when tracking iterates, else Omega only:
  // with a fixed iteration count only hdot_in is read back); X_ADJ_START:
  // the cotangent of hdot; X_ADJ_ACC / LAST: the running sum; X_ADJ_LAW: j
  const T* auxp = (OP == X_FWD || OP == X_ADJ_START || OP == X_ADJ_LAW)
                      ? A.in
                      : (OP == X_HIN ? A.warm : A.out);
  constexpr int NA = (NEED_AUX || OP == X_FWD) ? NC : 1;
  T aux[NA][2 * E];
  // one resource per component (each below 2 GiB); a null field reads zero
  auto field_rsrc = [&](const T* f, int cc) {
    return buffer_of(f ? f + (size_t)(c0 + cc) * csr : nullptr, f ? csr * sizeof(T) : 0);
  };
  if constexpr ((NEED_AUX || OP == X_FWD) && !PAIRED) {
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
      const __amdgpu_buffer_rsrc_t ra = field_rsrc(auxp, cc);
      const __amdgpu_buffer_rsrc_t r2 = field_rsrc(OP == X_FWD ? A.in2 : nullptr, cc);
#pragma unroll
      for (int e = 0; e < 2 * E; ++e) {
        bool need = valid && auxp != nullptr;
        if constexpr (OP == X_HIN) need = need && ch[e] == 0;
        const unsigned off = need ? (unsigned)((rowbase + 2 * (j + (e >> 1) * TPT) + (e & 1)) * sizeof(T)) : kBufMiss;
        aux[cc][e] = buffer_load_real<T>(ra, off);
        if constexpr (OP == X_FWD) aux[cc][e] += A.in2_coef * buffer_load_real<T>(r2, off);  // stage argument y + c k
      }
    }
  }
  if constexpr ((NEED_AUX || OP == X_FWD) && PAIRED) {
    bool need[2 * E];
#pragma unroll
    for (int e = 0; e < 2 * E; ++e) {
      bool nd = valid && auxp != nullptr;
      if constexpr (OP == X_HIN) nd = nd && ch[e] == 0;
      if constexpr (OP == X_UPDATE) nd = nd && (A.track || ch[e] != 0);
      if constexpr (OP == X_UPDATE_LAST) nd = nd && A.track;
      if constexpr (OP == X_ADJ_LAW) nd = nd && ch[e] != 0;     // j is read in Omega only
      need[e] = nd;
    }
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
      const __amdgpu_buffer_rsrc_t ra = field_rsrc(auxp, cc);
      const __amdgpu_buffer_rsrc_t r2 =
          field_rsrc((OP == X_FWD || OP == X_ADJ_START) ? A.in2 : nullptr, cc);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const unsigned off = (need[2 * m] || need[2 * m + 1])
                                 ? (unsigned)((rowbase + 2 * (j + m * TPT)) * sizeof(T))
                                 : kBufMiss;
        C2<T> v = buffer_load<T>(ra, off);
        if constexpr (OP == X_FWD) {  // stage argument y + c k (zero without in2)
          const C2<T> w = buffer_load<T>(r2, off);
          v.x += A.in2_coef * w.x;
          v.y += A.in2_coef * w.y;
        }
        if constexpr (OP == X_ADJ_START) {  // cotangent of hdot^K: lam + (1-chi) mu
          const C2<T> w = buffer_load<T>(r2, off);
          if (ch[2 * m] == 0) v.x += w.x;
          if (ch[2 * m + 1] == 0) v.y += w.y;
        }
        aux[cc][2 * m] = need[2 * m] ? v.x : T(0);
        aux[cc][2 * m + 1] = need[2 * m + 1] ? v.y : T(0);
      }
    }
  }


  if constexpr (HAS_INV) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if constexpr (LAZY) {
        if (c == 1) load_row(2);
      }
      // the kx = 0 slot holds X[0] + i X[M] (both real)
      const C2<T> xn = {Xs[c][0].y, T(0)};
      if (j == 0) Xs[c][0].y = T(0);
#pragma unroll
      for (int m = 0; m < E; ++m) lds.store(j + m * TPT, Xs[c][m]);
      if (j == 0) lds.store(M, xn);
      lds.sync();
      C2<T> Z[E];
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int k = j + m * TPT;
        const C2<T> pc = cconj(lds.load(M - k));                // conj X[M-k]
        const C2<T> ev = Xs[c][m] + pc;                          // X[k] + X[k+M]
        const C2<T> od = cmul(Xs[c][m] - pc, cconj(tw[k]));      // (X[k] - X[k+M]) w^-k
        Z[m] = {ev.x - od.y, ev.y + od.x};                       // ev + i od
      }
      lds.sync();
      fft_inverse<T, M, E>(Z, j, lds, tw, 2);
#pragma unroll
      for (int m = 0; m < E; ++m) {
        a[c][2 * m] = Z[m].x;
        a[c][2 * m + 1] = Z[m].y;
      }
    }
  }

  // ---- pointwise work on the nodes x = 2n, 2n+1, n = j + m TPT ----
  // real-field stores are collected (bit e: node e) and issued two nodes per access
  uint32_t st_out = 0, st_warm = 0;
  if constexpr (OP == X_LAW) {
    if (A.j_out && valid) {  // j itself, before the law (kept for the reverse mode)
      using T2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
#pragma unroll
      for (int m = 0; m < E; ++m)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          *reinterpret_cast<T2*>(A.j_out + c * csr + rowbase + 2 * (j + m * TPT)) = T2{a[c][2 * m], a[c][2 * m + 1]};
    }
  }
#pragma unroll
  for (int m = 0; m < E; ++m) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int x = 2 * (j + m * TPT) + h;
      const size_t idx = rowbase + x;
      const int e = 2 * m + h;
      const bool in = ch[NEED_CHI ? e : 0] != 0;
      if constexpr (OP == X_FWD) {
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) a[cc][e] = aux[cc][e];
      } else if constexpr (OP == X_LAW) {
        if (A.mom_partials && valid) {
          // moment readout of the state whose current this is: r x j, all nodes and Omega
          const double px = A.pos0[0] + A.step[0] * x;
          const double py = A.pos0[1] + A.step[1] * y;
          const double pz = A.pos0[2] + A.step[2] * z;
          const double jx = a[0][e], jy = a[1][e], jz = a[2][e];
          const double mx = py * jz - pz * jy, my = pz * jx - px * jz, mz = px * jy - py * jx;
          acc0 += mx;
          acc1 += my;
          acc2 += mz;
          if (in) {
            acc3 += mx;
            acc4 += my;
            acc5 += mz;
          }
        }
        if (in) {
          T lnk = A.kappa ? dev_log<T>(A.kappa[idx]) : T(0);
          if (A.hk_inv > T(0)) {  // e(j, h): the local field lowers the critical density
            T hs = T(0);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              T hc = A.in[c * csr + idx];
              if (A.in2) hc += A.in2_coef * A.in2[c * csr + idx];
              hs += hc * hc;
            }
            lnk -= A.kim_alpha * dev_log1p<T>(sqrt(hs) * A.hk_inv);
          }
          if (A.aniso)
            power_law_aniso<T>(a[0][e], a[1][e], a[2][e], A.aniso_w[0], A.aniso_w[1], A.aniso_w[2],
                               A.npow, lnk, A.expmax, clamps);
          else
            power_law<T>(a[0][e], a[1][e], a[2][e], A.npow, lnk, A.expmax, clamps);
        } else {
#pragma unroll
          for (int c = 0; c < 3; ++c) a[c][e] *= A.rho_out;
        }
      } else if constexpr (OP == X_HIN) {
        if (!in && A.warm) {
#pragma unroll
          for (int cc = 0; cc < NC; ++cc) a[cc][e] = aux[cc][e];
        }
        if (valid && (A.track || in)) {
          if constexpr (PAIRED) {
            st_out |= 1u << e;
          } else {
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) A.out[(c0 + cc) * csr + idx] = a[cc][e];
          }
        }
      } else if constexpr (OP == X_MASK) {
        if (!in) {
#pragma unroll
          for (int cc = 0; cc < NC; ++cc) a[cc][e] = T(0);
        }
      } else if constexpr (OP == X_UPDATE || OP == X_UPDATE_LAST) {
        T d2 = T(0);
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
          const T old = aux[cc][e];
          const T nw = in ? old : hdv[cc] + a[cc][e];
          const T dd = nw - old;
          d2 += dd * dd;
          a[cc][e] = nw;
        }
        if (valid && !in) {
          if (A.track) {
            acc0 += sqrt((double)d2);
            st_out |= 1u << e;
            if constexpr (OP == X_UPDATE_LAST) {
              if (A.warm_out) st_warm |= 1u << e;
            }
          } else if constexpr (OP == X_UPDATE_LAST) {
            st_out |= 1u << e;
            if (A.warm_out) st_warm |= 1u << e;
          }
        }
      } else if constexpr (OP == X_ADJ_START || OP == X_ADJ_ACC) {
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
          const T l = OP == X_ADJ_START ? aux[cc][e] : a[cc][e];
          if (valid) A.out[(c0 + cc) * csr + idx] = OP == X_ADJ_START ? l : aux[cc][e] + l;
          a[cc][e] = in ? T(0) : l;
        }
      } else if constexpr (OP == X_ADJ_LAST) {
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
          const T l0 = a[cc][e], cs = aux[cc][e];
          if (valid && A.warm_out) A.warm_out[(c0 + cc) * csr + idx] = in ? T(0) : l0;
          a[cc][e] = in ? cs + l0 : (A.warm_used ? T(0) : l0);
        }
        if (valid && !in) {
          acc0 += (double)aux[0][e];
          acc1 += (double)aux[1][e];
          acc2 += (double)aux[2][e];
        }
      } else if constexpr (OP == X_ADJ_LAW) {
        if (in) {
          const T jx = aux[0][e], jy = aux[1][e], jz = aux[2][e];
          const T ex = a[0][e], ey = a[1][e], ez = a[2][e];
          const T s = jx * jx + jy * jy + jz * jz;
          if (s > T(0)) {
            const T kap = A.kappa ? A.kappa[idx] : T(1);
            const T lnk = A.kappa ? dev_log<T>(kap) : T(0);
            const T lna = T(0.5) * dev_log<T>(s);
            T xp = (A.npow - T(1)) * (lna - lnk) - lnk;
            const bool clamped = xp > A.expmax;
            if (clamped) xp = A.expmax;
            const T rho = dev_exp<T>(xp);
            const T je = jx * ex + jy * ey + jz * ez;        // j . ebar
            // (de/dj)^T ebar = rho (ebar + (n-1) j (j . ebar) / |j|^2)
            const T q = clamped ? T(0) : (A.npow - T(1)) * je / s;
            a[0][e] = rho * (ex + q * jx);
            a[1][e] = rho * (ey + q * jy);
            a[2][e] = rho * (ez + q * jz);
            if (!clamped) {
              const double ee = (double)rho * (double)je;    // ebar . e
              acc0 += ee * (double)(lna - lnk);
              if (A.kappa_bar && valid) A.kappa_bar[idx] += -A.npow * (T)ee / kap;
            }
          } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) a[c][e] = T(0);
          }
        } else {
#pragma unroll
          for (int c = 0; c < 3; ++c) a[c][e] *= A.rho_out;
        }
      } else if constexpr (OP == X_STORE) {
        if (valid) st_out |= 1u << e;
      } else if constexpr (OP == X_MOMENT) {
        const bool use = valid && (!A.omega_only || in);
        if (use) {
          const double px = A.pos0[0] + A.step[0] * x;
          const double py = A.pos0[1] + A.step[1] * y;
          const double pz = A.pos0[2] + A.step[2] * z;
          const double jx = a[0][e], jy = a[1][e], jz = a[2][e];
          acc0 += py * jz - pz * jy;
          acc1 += pz * jx - px * jz;
          acc2 += px * jy - py * jx;
        }
      }
    }
  }

  if constexpr (OP == X_HIN || OP == X_UPDATE || OP == X_UPDATE_LAST || OP == X_STORE) {
    using T2 = typename std::conditional<sizeof(T) == 8, double2, float2>::type;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const unsigned bo = (st_out >> (2 * m)) & 3u, bw = (st_warm >> (2 * m)) & 3u;
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        const size_t ai = (c0 + cc) * csr + rowbase + 2 * (j + m * TPT);
        const T v0 = a[cc][2 * m], v1 = a[cc][2 * m + 1];
        if (bo == 3u) {
          *reinterpret_cast<T2*>(A.out + ai) = T2{v0, v1};
        } else if (bo) {
          if (bo & 1u) A.out[ai] = v0;
          if (bo & 2u) A.out[ai + 1] = v1;
        }
        if (bw == 3u) {
          *reinterpret_cast<T2*>(A.warm_out + ai) = T2{v0, v1};
        } else if (bw) {
          if (bw & 1u) A.warm_out[ai] = v0;
          if (bw & 2u) A.warm_out[ai + 1] = v1;
        }
      }
    }
  }

  if constexpr (OP == X_LAW) {
    if (A.mom_partials) {  // uniform across the block
      // fixed-order tree: lanes of each wavefront, then the wavefronts
      constexpr int NW = kBlock / 64;
      __shared__ double wsum[6 * NW];
      double v[6] = {acc0, acc1, acc2, acc3, acc4, acc5};
#pragma unroll
      for (int q = 0; q < 6; ++q) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
      }
      if ((tid & 63) == 0) {
#pragma unroll
        for (int q = 0; q < 6; ++q) wsum[q * NW + (tid >> 6)] = v[q];
      }
      __syncthreads();
      if (tid < 6) {
        double r = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) r += wsum[tid * NW + w];
        A.mom_partials[6 * blockIdx.x + tid] = r;
      }
    }
  }
  if (REDUCE && (OP == X_MOMENT || OP == X_ADJ_LAST || OP == X_ADJ_LAW || A.track)) {  // uniform
    red[tid] = acc0;
    red[kBlock + tid] = acc1;
    red[2 * kBlock + tid] = acc2;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
      if (tid < s) {
        red[tid] += red[tid + s];
        red[kBlock + tid] += red[kBlock + tid + s];
        red[2 * kBlock + tid] += red[2 * kBlock + tid + s];
      }
      __syncthreads();
    }
    if (tid == 0) {
      if constexpr (REDUCE3) {
        A.partials[3 * blockIdx.x + 0] = red[0];
        A.partials[3 * blockIdx.x + 1] = red[kBlock];
        A.partials[3 * blockIdx.x + 2] = red[2 * kBlock];
      } else {
        A.partials[blockIdx.x] = red[0];
      }
    }
  }
  if constexpr (OP == X_LAW) {
    if (clamps) atomicAdd(A.clamps, (unsigned long long)clamps);
  }

  if constexpr (HAS_FWD) {
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
      const int c = c0 + cc;
      C2<T> Z[E];
#pragma unroll
      for (int m = 0; m < E; ++m) Z[m] = {a[cc][2 * m], a[cc][2 * m + 1]};
      fft_forward<T, M, E>(Z, j, lds, tw, 2);
#pragma unroll
      for (int m = 0; m < E; ++m) lds.store(j + m * TPT, Z[m]);
      lds.sync();
#pragma unroll
      for (int m = 0; m < E; ++m) {
        const int k = j + m * TPT;
        const C2<T> pc = cconj(lds.load(k == 0 ? 0 : M - k));   // conj Z[M-k], Z[M] = Z[0]
        const C2<T> s = Z[m] + pc, d = Z[m] - pc;
        const C2<T> ev = {T(0.5) * s.x, T(0.5) * s.y};         // E[k]
        const C2<T> od = {T(0.5) * d.y, T(-0.5) * d.x};        // O[k] = d / (2i)
        C2<T> X = ev + cmul(tw[k], od);
        if (k == 0) X.y = Z[0].x - Z[0].y;                       // X[0] + i X[M]
        if (valid) P.main[c * csm + (size_t)rr * M + k] = X;
      }
      lds.sync();
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int N, int EMAX>
constexpr int tpt_of() {
  return N / elems_per_thread(N, EMAX);
}

template <typename T, int NX, int NC = 3, int OP = -1, int EV = 0>
static int xblocks_n(const Plan<T>& p) {
  constexpr int ROWS = kBlock / tpt_of<NX / 2, EV ? EV : ex_max<T, NC, OP>()>();
  const int rows = (p.r.xyhi - p.r.xylo) * (p.r.xzhi - p.r.xzlo);
  return (rows + ROWS - 1) / ROWS;
}

template <typename T>
int xpass_blocks(const Plan<T>& p) {
  switch (p.nx) {
    case 8: return xblocks_n<T, 8>(p);
    case 16: return xblocks_n<T, 16>(p);
    case 32: return xblocks_n<T, 32>(p);
    case 64: return xblocks_n<T, 64>(p);
    case 128: return xblocks_n<T, 128>(p);
    case 256: return xblocks_n<T, 256>(p);
    case 512: return xblocks_n<T, 512>(p);
    case 24: return xblocks_n<T, 24>(p);
    case 48: return xblocks_n<T, 48>(p);
    case 96: return xblocks_n<T, 96>(p);
    case 192: return xblocks_n<T, 192>(p);
  }
  return -1;
}

// the alternate bound of a per-component op: 4 where the default is 8 and
// the other way round
template <typename T, int OP>
constexpr int ex_alt() { return ex_max<T, 1, OP>() >= 8 ? 4 : 8; }

template <typename T, int NX, int OP, int NC, int EV = 0>
static void xlaunch_ev(const Plan<T>& p, const XArgs<T>& a, hipStream_t s, KTime t) {
  const int nb = xblocks_n<T, NX, NC, OP, EV>(p);
  if (nb <= 0) return;  // empty row range
  launch(xpass_kernel<T, NX, OP, NC, EV>, dim3(nb, NC == 3 ? 1 : 3, p.batch), dim3(kBlock), s, t, p, a);
}

template <typename T, int NX, int OP, int NC>
static void xlaunch_op(const Plan<T>& p, const XArgs<T>& a, hipStream_t s, KTime t) {
  if constexpr (NC == 1) {
    if (p.xalt) {
      xlaunch_ev<T, NX, OP, 1, ex_alt<T, OP>()>(p, a, s, t);
      return;
    }
  }
  xlaunch_ev<T, NX, OP, NC>(p, a, s, t);
}

template <typename T, int NX, int NC>
static hipError_t xlaunch_nc(const Plan<T>& p, int op, const XArgs<T>& a, hipStream_t s, KTime t) {
  switch (op) {
    case X_FWD: xlaunch_op<T, NX, X_FWD, NC>(p, a, s, t); break;
    case X_HIN: xlaunch_op<T, NX, X_HIN, NC>(p, a, s, t); break;
    case X_MASK: xlaunch_op<T, NX, X_MASK, NC>(p, a, s, t); break;
    case X_UPDATE: xlaunch_op<T, NX, X_UPDATE, NC>(p, a, s, t); break;
    case X_UPDATE_LAST: xlaunch_op<T, NX, X_UPDATE_LAST, NC>(p, a, s, t); break;
    case X_STORE: xlaunch_op<T, NX, X_STORE, NC>(p, a, s, t); break;
    case X_ADJ_START: xlaunch_op<T, NX, X_ADJ_START, NC>(p, a, s, t); break;
    case X_ADJ_ACC: xlaunch_op<T, NX, X_ADJ_ACC, NC>(p, a, s, t); break;
    default:
      if constexpr (NC == 3) {
        if (op == X_ADJ_LAST) {
          xlaunch_op<T, NX, X_ADJ_LAST, 3>(p, a, s, t);
          break;
        }
        if (op == X_ADJ_LAW) {
          xlaunch_op<T, NX, X_ADJ_LAW, 3>(p, a, s, t);
          break;
        }
        if (op == X_LAW) {
          xlaunch_op<T, NX, X_LAW, 3>(p, a, s, t);
          break;
        }
        if (op == X_MOMENT) {
          xlaunch_op<T, NX, X_MOMENT, 3>(p, a, s, t);
          break;
        }
      }
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Steps acting on one component at a time run one component per block
// (a third of the registers, more rows in flight).
template <typename T, int NX>
static hipError_t xlaunch_n(const Plan<T>& p, int op, const XArgs<T>& a, hipStream_t s, KTime t) {
  const bool per_component = op == X_FWD || op == X_HIN || op == X_MASK || op == X_STORE ||
                             op == X_ADJ_START || op == X_ADJ_ACC ||
                             ((op == X_UPDATE || op == X_UPDATE_LAST) && !a.track);
  return per_component ? xlaunch_nc<T, NX, 1>(p, op, a, s, t) : xlaunch_nc<T, NX, 3>(p, op, a, s, t);
}

template <typename T>
hipError_t launch_xpass(const Plan<T>& p, int op, const XArgs<T>& a, hipStream_t s, KTime t) {
  switch (p.nx) {
    case 8: return xlaunch_n<T, 8>(p, op, a, s, t);
    case 16: return xlaunch_n<T, 16>(p, op, a, s, t);
    case 32: return xlaunch_n<T, 32>(p, op, a, s, t);
    case 64: return xlaunch_n<T, 64>(p, op, a, s, t);
    case 128: return xlaunch_n<T, 128>(p, op, a, s, t);
    case 256: return xlaunch_n<T, 256>(p, op, a, s, t);
    case 512: return xlaunch_n<T, 512>(p, op, a, s, t);
    case 24: return xlaunch_n<T, 24>(p, op, a, s, t);
    case 48: return xlaunch_n<T, 48>(p, op, a, s, t);
    case 96: return xlaunch_n<T, 96>(p, op, a, s, t);
    case 192: return xlaunch_n<T, 192>(p, op, a, s, t);
  }
  return hipErrorInvalidValue;
}

template <typename T>
constexpr int ey_alt() { return ey_max<T>() >= 8 ? 4 : 8; }

template <typename T, int NY, int EV>
static hipError_t ylaunch_ev(const Plan<T>& p, bool inv, hipStream_t s, KTime t) {
  constexpr int EM = EV ? EV : ey_max<T>();
  constexpr int BLOCK = col_block<T, NY, EM>();
  constexpr int COLS = BLOCK / tpt_of<NY, EM>();
  const int M = p.nx / 2;
  const int nzr = p.r.zhi - p.r.zlo;
  if (nzr <= 0) return hipSuccess;  // nothing to transform
  const int ncm = 3 * nzr * M;
  const dim3 grid((ncm + COLS - 1) / COLS, 1, p.batch), block(BLOCK);
  if (inv)
    launch(ypass_kernel<T, NY, true, EV>, grid, block, s, t, p.main, M, p.nz, p.r, p.ay.tw, p.stop, p.zs_main);
  else
    launch(ypass_kernel<T, NY, false, EV>, grid, block, s, t, p.main, M, p.nz, p.r, p.ay.tw, p.stop, p.zs_main);
  return hipGetLastError();
}

template <typename T, int NY>
static hipError_t ylaunch_n(const Plan<T>& p, bool inv, hipStream_t s, KTime t) {
  return p.yalt ? ylaunch_ev<T, NY, ey_alt<T>()>(p, inv, s, t) : ylaunch_ev<T, NY, 0>(p, inv, s, t);
}

template <typename T>
hipError_t launch_ypass(const Plan<T>& p, bool inv, hipStream_t s, KTime t) {
  switch (p.ny) {
    case 8: return ylaunch_n<T, 8>(p, inv, s, t);
    case 16: return ylaunch_n<T, 16>(p, inv, s, t);
    case 32: return ylaunch_n<T, 32>(p, inv, s, t);
    case 64: return ylaunch_n<T, 64>(p, inv, s, t);
    case 128: return ylaunch_n<T, 128>(p, inv, s, t);
    case 256: return ylaunch_n<T, 256>(p, inv, s, t);
    case 512: return ylaunch_n<T, 512>(p, inv, s, t);
    case 24: return ylaunch_n<T, 24>(p, inv, s, t);
    case 48: return ylaunch_n<T, 48>(p, inv, s, t);
    case 96: return ylaunch_n<T, 96>(p, inv, s, t);
    case 192: return ylaunch_n<T, 192>(p, inv, s, t);
  }
  return hipErrorInvalidValue;
}

template <typename T>
constexpr int ez_alt() { return ez_max<T>() >= 8 ? 4 : 8; }

template <typename T, int NZ, int EV>
static hipError_t zlaunch_ev(const Plan<T>& p, int sym, T coef, hipStream_t s, KTime t) {
  constexpr int BLOCK = z_block<T, NZ, EV>();
  constexpr int COLS = BLOCK / tpt_of<NZ, EV ? EV : ez_max<T>()>();
  const int M = p.nx / 2;
  const dim3 grid((p.ny * M + COLS - 1) / COLS, 1, p.batch), block(BLOCK);
  switch (sym) {
    case Z_CURL:
      launch(zpass_kernel<T, NZ, Z_CURL, EV>, grid, block, s, t, p.main, p.ny, M, p.ax, p.ay, p.az, coef,
             p.r, p.stop, p.zs_main);
      break;
    case Z_PHI:
      launch(zpass_kernel<T, NZ, Z_PHI, EV>, grid, block, s, t, p.main, p.ny, M, p.ax, p.ay, p.az, coef,
             p.r, p.stop, p.zs_main);
      break;
    case Z_PHI_SMOOTH:
      launch(zpass_kernel<T, NZ, Z_PHI_SMOOTH, EV>, grid, block, s, t, p.main, p.ny, M, p.ax, p.ay,
             p.az, coef, p.r, p.stop, p.zs_main);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int NZ>
static hipError_t zlaunch_n(const Plan<T>& p, int sym, T coef, hipStream_t s, KTime t) {
  return p.zalt ? zlaunch_ev<T, NZ, ez_alt<T>()>(p, sym, coef, s, t) : zlaunch_ev<T, NZ, 0>(p, sym, coef, s, t);
}

template <typename T>
hipError_t launch_zpass(const Plan<T>& p, int sym, T coef, hipStream_t s, KTime t) {
  switch (p.nz) {
    case 8: return zlaunch_n<T, 8>(p, sym, coef, s, t);
    case 16: return zlaunch_n<T, 16>(p, sym, coef, s, t);
    case 32: return zlaunch_n<T, 32>(p, sym, coef, s, t);
    case 64: return zlaunch_n<T, 64>(p, sym, coef, s, t);
    case 128: return zlaunch_n<T, 128>(p, sym, coef, s, t);
    case 256: return zlaunch_n<T, 256>(p, sym, coef, s, t);
    case 512: return zlaunch_n<T, 512>(p, sym, coef, s, t);
    case 24: return zlaunch_n<T, 24>(p, sym, coef, s, t);
    case 48: return zlaunch_n<T, 48>(p, sym, coef, s, t);
    case 96: return zlaunch_n<T, 96>(p, sym, coef, s, t);
    case 192: return zlaunch_n<T, 192>(p, sym, coef, s, t);
  }
  return hipErrorInvalidValue;
}

template int xpass_blocks<double>(const Plan<double>&);
template int xpass_blocks<float>(const Plan<float>&);
template hipError_t launch_xpass<double>(const Plan<double>&, int, const XArgs<double>&, hipStream_t,
                                         KTime);
template hipError_t launch_xpass<float>(const Plan<float>&, int, const XArgs<float>&, hipStream_t,
                                        KTime);
template hipError_t launch_ypass<double>(const Plan<double>&, bool, hipStream_t, KTime);
template hipError_t launch_ypass<float>(const Plan<float>&, bool, hipStream_t, KTime);
template hipError_t launch_zpass<double>(const Plan<double>&, int, double, hipStream_t, KTime);
template hipError_t launch_zpass<float>(const Plan<float>&, int, float, hipStream_t, KTime);

}  // namespace scfft
