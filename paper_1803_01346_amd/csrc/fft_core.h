// Device FFT engine for gfx950: Stockham radix passes on data held in
// registers, exchanged through LDS between passes.
//
// A length-N transform is owned by TPT = N / E threads; thread j of a
// transform holds the E elements v[m] = x[j + m * TPT], m = 0..E-1, both on
// entry and on exit (natural order, no bit reversal).  Each Stockham pass of
// radix R (R divides E) lets thread j run E/R butterflies b = j + q * TPT,
// whose inputs are x[b + r * N/R] = v[q + r * E/R]; outputs go to
// (b / Ns) * Ns * R + (b % Ns) + r * Ns, where Ns is the product of earlier
// radices.  After the last pass that position is again v[q + r * E/R], so
// the final pass needs no exchange.
//
// Lengths are powers of two or three times a power of two.
//
// Forward transforms use exp(-2 pi i k / N) (the paper's sign, Sec. 2 text
// before Eq. 7); the inverse is conj(forward(conj(x))), unnormalised.
#pragma once

#include <hip/hip_runtime.h>

namespace scfft {

template <typename T>
struct C2 {
  T x, y;
};

template <typename T>
__device__ __forceinline__ C2<T> operator+(C2<T> a, C2<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ C2<T> operator-(C2<T> a, C2<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ C2<T> cconj(C2<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ C2<T> cscale(C2<T> a, T s) { return {a.x * s, a.y * s}; }

// ---- in-register DFTs of radix 2, 3, 4, 8 (forward sign) ----

template <typename T>
__device__ __forceinline__ void dft2(C2<T>* v) {
  C2<T> a = v[0];
  v[0] = a + v[1];
  v[1] = a - v[1];
}

template <typename T>
__device__ __forceinline__ void dft4(C2<T>& a, C2<T>& b, C2<T>& c, C2<T>& d) {
  C2<T> t0 = a + c, t1 = a - c, t2 = b + d, t3 = b - d;
  a = t0 + t2;
  c = t0 - t2;
  b = {t1.x + t3.y, t1.y - t3.x};  // t1 - i t3
  d = {t1.x - t3.y, t1.y + t3.x};  // t1 + i t3
}

template <typename T>
__device__ __forceinline__ void dft4(C2<T>* v) { dft4(v[0], v[1], v[2], v[3]); }

template <typename T>
__device__ __forceinline__ void dft8(C2<T>* v) {
  const T r = T(0.70710678118654752440084436210484904);
  C2<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  C2<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  // twiddles w8^k o_k, w8 = exp(-i pi / 4)
  C2<T> t1 = {(o1.x + o1.y) * r, (o1.y - o1.x) * r};
  C2<T> t2 = {o2.y, -o2.x};
  C2<T> t3 = {(o3.y - o3.x) * r, -(o3.y + o3.x) * r};
  v[0] = e0 + o0;
  v[4] = e0 - o0;
  v[1] = e1 + t1;
  v[5] = e1 - t1;
  v[2] = e2 + t2;
  v[6] = e2 - t2;
  v[3] = e3 + t3;
  v[7] = e3 - t3;
}

// w3 = exp(-2 pi i / 3) = -1/2 - i sqrt(3)/2:
//   y0 = a + (b + c),  y1,2 = a - (b + c)/2 -/+ i sqrt(3)/2 (b - c)
template <typename T>
__device__ __forceinline__ void dft3(C2<T>* v) {
  const T h = T(0.86602540378443864676372317075293618);
  const C2<T> s = v[1] + v[2], d = v[1] - v[2];
  const C2<T> m = {v[0].x - T(0.5) * s.x, v[0].y - T(0.5) * s.y};
  const C2<T> r = {h * d.y, -h * d.x};  // -i sqrt(3)/2 (b - c)
  v[0] = v[0] + s;
  v[1] = m + r;
  v[2] = m - r;
}

template <typename T, int R>
__device__ __forceinline__ void dftR(C2<T>* v) {
  if constexpr (R == 2) dft2(v);
  else if constexpr (R == 3) dft3(v);
  else if constexpr (R == 4) dft4(v);
  else if constexpr (R == 8) dft8(v);
  else static_assert(R == 2 || R == 3 || R == 4 || R == 8, "radix");
}

// ---- pass plan: radices for length N with E elements per thread ----

// Lengths are 2^k or 3 * 2^k.  A length 3 * 2^k runs one radix-3 pass and
// then radix-2^j passes; its threads hold 3 * E2 elements, E2 = emax / 2
// (at least 2, at most the power-of-two factor), so that 3 and every later
// radix divide E.
__host__ __device__ constexpr int elems_per_thread(int n, int emax = 8) {
  if (n % 3 == 0) {
    int e2 = emax / 2 < 2 ? 2 : emax / 2;
    if (e2 > n / 3) e2 = n / 3;
    return 3 * e2;
  }
  return n >= emax ? emax : n;
}

// radix of pass p (0-based) for length N with E per thread: for 3 * 2^k a
// radix-3 pass first; then E (E / 3) while the remaining factor allows, then
// the remainder.
__host__ __device__ constexpr int pass_radix(int n, int e, int p) {
  if (n % 3 == 0) {
    if (p == 0) return 3;
    n /= 3;
    e /= 3;
    --p;
  }
  int rem = n;
  for (int i = 0; i < p; ++i) rem /= (rem >= e ? e : rem);
  return rem >= e ? e : rem;
}
__host__ __device__ constexpr int pass_count(int n, int e) {
  int c = 0;
  if (n % 3 == 0) {
    n /= 3;
    e /= 3;
    c = 1;
  }
  for (int rem = n; rem > 1; rem /= (rem >= e ? e : rem)) ++c;
  return c;
}
__host__ __device__ constexpr int pass_span(int n, int e, int p) {  // Ns of pass p
  int ns = 1;
  for (int i = 0; i < p; ++i) ns *= pass_radix(n, e, i);
  return ns;
}

// One Stockham pass.  tw points at a table of exp(-2 pi i k / (N * TWS)),
// k = 0 .. N*TWS - 1, read with stride TWS.  Lds provides store(idx, v),
// load(idx) for this transform and sync().
template <typename T, int N, int E, int P, class Lds>
__device__ __forceinline__ void stockham_pass(C2<T> (&v)[E], int j, Lds& lds,
                                              const C2<T>* __restrict__ tw, int tws) {
  constexpr int R = pass_radix(N, E, P);
  constexpr int NS = pass_span(N, E, P);
  constexpr int TPT = N / E;
  constexpr int Q = E / R;
  constexpr bool LAST = (P + 1 == pass_count(N, E));
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int b = j + q * TPT;
    C2<T> a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) a[r] = v[q + r * Q];
    const int kk = b % NS;
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) a[r] = cmul(a[r], tw[(r * kk * (N / (NS * R))) * tws]);
    }
    dftR<T, R>(a);
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[q + r * Q] = a[r];
    } else {
      const int base = (b / NS) * NS * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) lds.store(base + r * NS, a[r]);
    }
  }
  if constexpr (!LAST) {
    lds.sync();
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = lds.load(j + m * TPT);
    lds.after_load();
  }
}

template <typename T, int N, int E, int P, class Lds>
__device__ __forceinline__ void fft_passes(C2<T> (&v)[E], int j, Lds& lds,
                                           const C2<T>* __restrict__ tw, int tws) {
  if constexpr (P < pass_count(N, E)) {
    stockham_pass<T, N, E, P>(v, j, lds, tw, tws);
    fft_passes<T, N, E, P + 1>(v, j, lds, tw, tws);
  }
}

// Forward (exp(-i...)) transform of length N; all threads of the block must
// call it together (it synchronises the block between passes).
template <typename T, int N, int E, class Lds>
__device__ __forceinline__ void fft_forward(C2<T> (&v)[E], int j, Lds& lds,
                                            const C2<T>* __restrict__ tw, int tws) {
  fft_passes<T, N, E, 0>(v, j, lds, tw, tws);
}

template <typename T, int N, int E, class Lds>
__device__ __forceinline__ void fft_inverse(C2<T> (&v)[E], int j, Lds& lds,
                                            const C2<T>* __restrict__ tw, int tws) {
#pragma unroll
  for (int m = 0; m < E; ++m) v[m].y = -v[m].y;
  fft_passes<T, N, E, 0>(v, j, lds, tw, tws);
#pragma unroll
  for (int m = 0; m < E; ++m) v[m].y = -v[m].y;
}

// Twiddle table of one axis staged in LDS.  Every pass of a transform after
// the first reads it; from global memory (an L2 round trip per pass) that
// latency sat between the LDS exchanges.  fetch() issues the global loads
// (before the block's other loads, so waiting for them later waits for
// nothing else); put() writes the LDS copy.  The copy must be visible to the
// whole block before the first read: with column layouts every exchange is a
// block barrier and the first pass of a transform reads no twiddle, so put()
// before the first transform suffices; with row layouts (wavefront-local
// exchanges) the caller adds one block barrier after put().
template <typename T, int N, int BLOCK>
struct LdsTwiddles {
  // at most two entries per thread, held as plain scalars (a C2 or an array
  // member is placed in LDS by the compiler's alloca promotion)
  static_assert(N <= 2 * BLOCK, "twiddle table larger than two entries per thread");
  T r0x = T(0), r0y = T(0), r1x = T(0), r1y = T(0);
  __device__ __forceinline__ void fetch(const C2<T>* __restrict__ g) {
    const int i = (int)threadIdx.x;
    if (i < N) {
      const C2<T> w = g[i];
      r0x = w.x;
      r0y = w.y;
    }
    if (N > BLOCK && i + BLOCK < N) {
      const C2<T> w = g[i + BLOCK];
      r1x = w.x;
      r1y = w.y;
    }
  }
  __device__ __forceinline__ void put(C2<T>* s) const {
    const int i = (int)threadIdx.x;
    if (i < N) s[i] = C2<T>{r0x, r0y};
    if (N > BLOCK && i + BLOCK < N) s[i + BLOCK] = C2<T>{r1x, r1y};
  }
};

// LDS layouts.  Column-major: COLS transforms side by side, element idx of
// column c at idx * COLS + c (lanes of one row of columns are contiguous).
//
// Each layout provides sync() (between the stores of a pass and the loads of
// the next) and after_load() (before the next pass may store again).
template <typename T, int COLS>
struct LdsCols {
  C2<T>* base;
  int col;
  __device__ __forceinline__ void store(int idx, C2<T> v) { base[idx * COLS + col] = v; }
  __device__ __forceinline__ C2<T> load(int idx) const { return base[idx * COLS + col]; }
  __device__ __forceinline__ void sync() { __syncthreads(); }
  __device__ __forceinline__ void after_load() { __syncthreads(); }
};

// Column-major with two buffers of N * COLS elements used alternately:
// consecutive exchanges never touch the same buffer, so one block barrier
// per exchange suffices (the barrier of exchange p+1 also orders the loads
// of exchange p before the stores of exchange p+2).  The parity carries
// over from one transform to the next.
template <typename T, int N, int COLS>
struct LdsColsPP {
  C2<T>* base;
  int col;
  int off = 0;
  __device__ __forceinline__ void store(int idx, C2<T> v) { base[off + idx * COLS + col] = v; }
  __device__ __forceinline__ C2<T> load(int idx) const { return base[off + idx * COLS + col]; }
  __device__ __forceinline__ void sync() { __syncthreads(); }
  __device__ __forceinline__ void after_load() { off = off ? 0 : N * COLS; }
};

// Barrier among the lanes of one wavefront: orders this wave's LDS stores
// before its later LDS loads (a wave's LDS operations execute in order; the
// fences keep the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row-major, rows of STRIDE elements holding indices 0..N inclusive, with
// an XOR swizzle inside each block of 8 elements: bits 0..2 of the index are
// XORed with parities of bits 3..6 (masks 3, 5, 3), chosen by a search over
// all such linear swizzles for the fewest bank conflicts of the split and
// Stockham exchanges of one row (32 four-byte banks, 16-byte elements, eight
// lanes per cycle).  Contiguous accesses stay permutations; the strided
// stores of the radix-4 passes spread over the banks.  When several rows
// share a lane group (N/E < 16) the row index joins the high bits.  When the
// N/E threads of a row lie in one wavefront (N/E <= 64, rows aligned to
// waves) the exchange needs only a wavefront barrier.
template <typename T, int N, int E>
struct LdsRows {
  static constexpr int STRIDE = ((N + 1 + 15) / 16) * 16;
  static constexpr bool ROWMIX = (N / E) < 16;
  static constexpr bool IN_WAVE = (N / E) <= 64;
  C2<T>* base;
  int row;
  __device__ __forceinline__ static int parity(int v) { return __builtin_popcount(v) & 1; }
  __device__ __forceinline__ int swz(int idx) const {
    const int h = ((idx >> 3) + (ROWMIX ? 2 * row : 0)) & 15;
    return idx ^ (parity(h & 3) | (parity(h & 5) << 1) | (parity(h & 3) << 2));
  }
  __device__ __forceinline__ void store(int idx, C2<T> v) { base[row * STRIDE + swz(idx)] = v; }
  __device__ __forceinline__ C2<T> load(int idx) const { return base[row * STRIDE + swz(idx)]; }
  __device__ __forceinline__ void sync() {
    if constexpr (IN_WAVE)
      wave_sync();
    else
      __syncthreads();
  }
  __device__ __forceinline__ void after_load() { sync(); }
};

// ---- column transform with lane-swapped index bits (gfx950) ----
//
// A column of N = 2^n points held by TPT = N / E lanes, E = 2^RB elements
// each, in a block whose lane index is j * COLS + column (COLS = 8 or 16, so
// the low JL = 3 or 2 bits of j sit in lane bits 3..5 or 4..5 and the rest of
// j selects the wavefront).  The transform is a decimation-in-frequency FFT
// taken as steps over groups of index bits, each step a radix-2^b DFT over
// bits that a lane holds in its registers, followed by its twiddles:
//   step 1: the top RB bits (radix E);
//   lane swaps: the two bits on lane bits 5 and 4 trade places with register
//     bits RB-1 and RB-2 (v_permlane32_swap / v_permlane16_swap, a 2 x 2
//     transpose of two registers across two halves of the lane range);
//   step 2: those two bits (radix 4);
//   one LDS exchange: the remaining P2 low bits (held by the wavefront index
//     and, with 8 columns, lane bit 3) move to the top register bits and,
//     where RB < P2, lane bits 5 and 4;
//   step 3: radix 2^B3 over the register bits; where B4 = P2 - B3 > 0, lane
//     swaps once more and step 4 (radix 2^B4, no twiddles).
// A step over index bits [s, s + b) of a length-L sub-transform leaves its
// output digit k in those bits, times w_L^(lo k) with lo the index bits below
// s; digits come out lowest first, so the frequency of the element at final
// position z is read off its bit fields (freq()).  The output stays in that
// order; the inverse runs the transposed steps in reverse order (twiddles
// before each DFT, decimation in time), conjugated on entry and exit, and
// returns to natural order, so a pointwise product between the two needs no
// reordering.  Against the Stockham passes (three LDS round trips per
// 128-point transform with four elements per lane) this takes one.
__host__ __device__ constexpr int ilog2_exact(int x) {
  int r = 0;
  while ((1 << r) < x) ++r;
  return (1 << r) == x ? r : -1;
}

template <typename T, int N, int E, int COLS>
struct LaneCol {
  static constexpr int n = ilog2_exact(N), RB = ilog2_exact(E), JL = 6 - ilog2_exact(COLS);
  static constexpr int WB = n - RB - JL;  // j bits above the lane bits (wavefront index)
  static constexpr int P2 = WB + JL - 2;  // index bits left for the steps after the exchange
  static constexpr int B3 = RB < P2 ? RB : P2, B4 = P2 - B3;
  static constexpr bool ok = n > 0 && (E == 4 || E == 8) && (COLS == 8 || COLS == 16) && WB >= 0 &&
                             P2 >= 1 && B4 <= 2;

  __device__ __forceinline__ static int jb(int j, int b) { return (j >> b) & 1; }
  __device__ __forceinline__ static int l4(int j) { return jb(j, JL - 2); }  // j bit on lane bit 4
  __device__ __forceinline__ static int l5(int j) { return jb(j, JL - 1); }  // j bit on lane bit 5
  // natural index of element m of lane j (load and store order)
  __device__ __forceinline__ static int pos_a(int j, int m) {
    return (m << (n - RB)) + ((j & ((1 << JL) - 1)) << WB) + (j >> JL);
  }
  // index held by (j, m) after the first lane swaps
  __device__ __forceinline__ static int pos_a2(int j, int m) {
    int z = (((m >> (RB - 1)) & 1) << (P2 + 1)) | (((m >> (RB - 2)) & 1) << P2);
    if constexpr (RB > 2) z |= (m & ((1 << (RB - 2)) - 1)) << (n - RB);
    z |= (l5(j) << (n - 1)) | (l4(j) << (n - 2)) | (j >> JL);
    if constexpr (JL == 3) z |= (j & 1) << WB;
    return z;
  }
  // lane-bit part of the indices after the exchange (the low B4 bits)
  __device__ __forceinline__ static int lrem(int j) {
    return B4 == 1 ? l5(j) : (B4 == 2 ? 2 * l5(j) + l4(j) : 0);
  }
  // index held by (j, m) after the exchange: the finished top RB + 2 bits F
  // come from the wavefront index, lane bit 3, the lane bits and register
  // bits the last steps leave free
  __device__ __forceinline__ static int pos_b(int j, int m) {
    int f = j >> JL, w = WB;
    if constexpr (JL == 3) { f |= (j & 1) << w; w += 1; }
    if constexpr (B4 == 0) { f |= (l4(j) << w) | (l5(j) << (w + 1)); w += 2; }
    if constexpr (B4 == 1) { f |= l4(j) << w; w += 1; }
    if constexpr (RB > B3) f |= (m & ((1 << (RB - B3)) - 1)) << w;
    return (f << P2) + ((m >> (RB - B3)) << (P2 - B3)) + lrem(j);
  }
  // frequency of the element (j, m) after the forward transform
  __device__ __forceinline__ static int freq(int j, int m) {
    int jj = j, mm = m;
    if constexpr (B4 >= 1) {
      jj = (jj & ~(1 << (JL - 1))) | (((m >> (RB - 1)) & 1) << (JL - 1));
      mm = (mm & ~(1 << (RB - 1))) | (l5(j) << (RB - 1));
    }
    if constexpr (B4 == 2) {
      jj = (jj & ~(1 << (JL - 2))) | (((m >> (RB - 2)) & 1) << (JL - 2));
      mm = (mm & ~(1 << (RB - 2))) | (l4(j) << (RB - 2));
    }
    const int z = pos_b(jj, mm);
    return (z >> (n - RB)) + E * ((z >> P2) & 3) + 4 * E * ((z >> (P2 - B3)) & ((1 << B3) - 1)) +
           4 * E * (1 << B3) * (z & ((1 << B4) - 1));
  }

  // 2 x 2 transpose of registers x, y across lane bit LB (4 or 5): lanes with
  // the bit clear keep x and take the partner's x into y; lanes with it set
  // keep y and take the partner's y into x
  template <int LB>
  __device__ __forceinline__ static void swap_words(unsigned& x, unsigned& y) {
    if constexpr (LB == 5) {
      const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
      x = r[0];
      y = r[1];
    } else {
      const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
      x = r[0];
      y = r[1];
    }
  }
  template <int LB>
  __device__ __forceinline__ static void swap_pair(C2<T>& x, C2<T>& y) {
    struct Words { unsigned w[sizeof(C2<T>) / 4]; };
    Words a = __builtin_bit_cast(Words, x), b = __builtin_bit_cast(Words, y);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(C2<T>) / 4); ++i) swap_words<LB>(a.w[i], b.w[i]);
    x = __builtin_bit_cast(C2<T>, a);
    y = __builtin_bit_cast(C2<T>, b);
  }
  // lane bit LB <-> register bit RBIT
  template <int LB, int RBIT>
  __device__ __forceinline__ static void swap_bit(C2<T> (&v)[E]) {
#pragma unroll
    for (int m = 0; m < E; ++m)
      if (((m >> RBIT) & 1) == 0) swap_pair<LB>(v[m], v[m | (1 << RBIT)]);
  }

  // DFT over register bits [SH, SH + B) with twiddles tw[lo * k] on output k
  // (PRE: on input k, the transposed step)
  template <int SH, int B, bool PRE, bool TW>
  __device__ __forceinline__ static void step(C2<T> (&v)[E], const C2<T>* tw, int lo) {
    constexpr int R = 1 << B;
#pragma unroll
    for (int o = 0; o < E; ++o) {
      if (((o >> SH) & (R - 1)) != 0) continue;
      C2<T> a[R];
#pragma unroll
      for (int d = 0; d < R; ++d) a[d] = v[o | (d << SH)];
      if constexpr (TW && PRE) {
#pragma unroll
        for (int k = 1; k < R; ++k) a[k] = cmul(a[k], tw[lo * k]);
      }
      dftR<T, R>(a);
      if constexpr (TW && !PRE) {
#pragma unroll
        for (int k = 1; k < R; ++k) a[k] = cmul(a[k], tw[lo * k]);
      }
#pragma unroll
      for (int k = 0; k < R; ++k) v[o | (k << SH)] = a[k];
    }
  }

  // buf: this transform's LDS buffer (N * COLS elements); the caller
  // alternates two buffers between transforms, so each exchange needs one
  // block barrier.  tw: exp(-2 pi i k / N), k < N, readable by the block.
  __device__ __forceinline__ static void exchange_ab(C2<T> (&v)[E], int j, int col, C2<T>* buf, bool to_b) {
#pragma unroll
    for (int m = 0; m < E; ++m) buf[(to_b ? pos_a2(j, m) : pos_b(j, m)) * COLS + col] = v[m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = buf[(to_b ? pos_b(j, m) : pos_a2(j, m)) * COLS + col];
  }
  __device__ __forceinline__ static void forward(C2<T> (&v)[E], int j, int col, C2<T>* buf, const C2<T>* tw) {
    static_assert(ok, "shape outside the lane-swapped layout (use the Stockham passes)");
    const int lo2 = ((j & ((1 << (JL - 2)) - 1)) << WB) + (j >> JL);
    step<0, RB, false, true>(v, tw, pos_a(j, 0));
    swap_bit<5, RB - 1>(v);
    swap_bit<4, RB - 2>(v);
    step<RB - 2, 2, false, true>(v, tw, lo2 * E);
    exchange_ab(v, j, col, buf, true);
    step<RB - B3, B3, false, (B4 > 0)>(v, tw, lrem(j) * 4 * E);
    if constexpr (B4 >= 1) swap_bit<5, RB - 1>(v);
    if constexpr (B4 == 2) swap_bit<4, RB - 2>(v);
    if constexpr (B4 >= 1) step<RB - B4, B4, false, false>(v, tw, 0);
  }
  __device__ __forceinline__ static void inverse(C2<T> (&v)[E], int j, int col, C2<T>* buf, const C2<T>* tw) {
    static_assert(ok, "shape outside the lane-swapped layout (use the Stockham passes)");
    const int lo2 = ((j & ((1 << (JL - 2)) - 1)) << WB) + (j >> JL);
#pragma unroll
    for (int m = 0; m < E; ++m) v[m].y = -v[m].y;
    if constexpr (B4 >= 1) step<RB - B4, B4, true, false>(v, tw, 0);
    if constexpr (B4 == 2) swap_bit<4, RB - 2>(v);
    if constexpr (B4 >= 1) swap_bit<5, RB - 1>(v);
    step<RB - B3, B3, true, (B4 > 0)>(v, tw, lrem(j) * 4 * E);
    exchange_ab(v, j, col, buf, false);
    step<RB - 2, 2, true, true>(v, tw, lo2 * E);
    swap_bit<4, RB - 2>(v);
    swap_bit<5, RB - 1>(v);
    step<0, RB, true, true>(v, tw, pos_a(j, 0));
#pragma unroll
    for (int m = 0; m < E; ++m) v[m].y = -v[m].y;
  }
};

}  // namespace scfft
