// Launch shapes of the transform passes: one table of compile-time constants,
// each chosen by measurement on MI355X (gfx950).  The run-time alternates of
// the per-component X, the Y and the Z passes (rhs options x_alt, y_alt,
// z_alt) are other instantiations of the same kernels, picked per grid by
// scfft_autotune.
#pragma once

namespace scfft {
namespace tune {

// Elements per thread (an upper bound; also the largest radix) of one line.
constexpr int kEx3F64 = 4;     // X passes holding all three components (power law, moment,
constexpr int kEx3F32 = 4;     //   adaptive update, reverse mode)
constexpr int kEx1F64 = 4;     // per-component X passes (input, warm start, masks, updates,
constexpr int kEx1F32 = 4;     //   store, reverse mode): shorter lines, more rows per block
constexpr int kEyF64 = 4;      // Y passes (one component per column); FP64: 8 lanes of a
constexpr int kEyF32 = 8;      //   16 KB tile hold 8 blocks per CU (4 with 8 elements)
constexpr int kEzF64 = 4;      // Z passes (three components of a column in registers)
constexpr int kEzF32 = 8;

// Column passes exchange through two alternating LDS buffers (one barrier per
// exchange) where that does not cost occupancy: the Z pass; the Y pass keeps
// one buffer (two would halve its blocks per CU).
constexpr bool kPingPongY = false;
constexpr bool kPingPongZ = true;

// Threads per block of a column pass: 256, doubled while the columns of one
// block span fewer than this many contiguous bytes of a row.  The FP32 Z
// pass stops at 64 bytes: a 512-thread block would hold 143 VGPRs per lane
// and leave one block per CU (measured slower at 256^3).
constexpr int kColBytes = 128;
constexpr int kColBytesZF64 = 128;
constexpr int kColBytesZF32 = 64;

// Threads per block of the fused xy-plane pass (one block per plane): FP64
// lines need more registers, so FP64 uses fewer, fuller threads.
constexpr int kXYBlockF64 = 512;
constexpr int kXYBlockF32 = 1024;

}  // namespace tune
}  // namespace scfft
