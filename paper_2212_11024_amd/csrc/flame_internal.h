// Host-side context and launcher declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <string>

#include "../../include/flame.h"
#include "flame_device.h"

struct flame_ctx {
  flame_params p{};
  int device = 0;
  hipStream_t stream = nullptr;
  size_t n = 0;              // nodes
  size_t stride = 0;         // elements between consecutive population arrays
  void* storage = nullptr;   // caller-owned populations
  int parity = 0;            // AA in-place sets: 0 = canonical slots, 1 = swapped slots
  int cur = 0;               // two-lattice sets: index of the copy holding the current state
  int64_t steps = 0;
  double frest[27]{};        // f^mhd(0)(1, 0, b0)
  double omega = 0, omega_b = 0;
  double cfl = 0;
  // launch shape (tuning; read from the environment at flame_init, results do not depend on it):
  // planes per workgroup of the stencil kernel (0: the built-in 32) and threads per row block of
  // the node-local kernels (0: the row rounded up to whole wavefronts, at most 256)
  int zchunk = 0;
  int row_tx = 0;
  bool global_addr = false;   // FLAME_GLOBAL_ADDRESSING=1: no buffer addressing in the step
  std::string err;
  // library-owned scratch
  double* red_partials = nullptr;
  int red_blocks = 0;
  double* scratch = nullptr;   // this device's static reduction scratch (not owned)
  double* spec_real = nullptr;
  void* spec_cplx = nullptr;
  double* spec_partials = nullptr;
  int spec_blocks = 0;
  int spec_nshells = 0;
  hipfftHandle plan{};
  bool plan_ok = false;
  hipfftHandle plan_inv{};   // complex-to-real inverse, for spectral derivatives
  bool plan_inv_ok = false;
};

namespace flame {

// Pointers to the population sets of the current step.
struct SetPtrs {
  void* f_src;
  void* f_dst;
  void* g_src;
  void* g_dst;
  bool fluid_aa;     // fluid set updated in place (else two-lattice pull)
  bool mag_aa;       // magnetic set updated in place (else two-lattice pull)
};

inline size_t value_bytes(int storage) { return storage == FLAME_F64 ? 8 : storage == FLAME_F32 ? 4 : 2; }

// Population arrays are laid out back to back with a stride of the node count rounded up to
// 256 bytes plus a pad, so that the 48 arrays do not all start at large powers of two apart.
#ifndef FLAME_STRIDE_PAD_BYTES
#define FLAME_STRIDE_PAD_BYTES 0
#endif
inline size_t population_stride(const flame_params& p) {
  const size_t vb = value_bytes(p.storage);
  const size_t n = static_cast<size_t>(p.nx) * p.ny * p.nz;
  const size_t align = 256 / vb;
  return (n + align - 1) / align * align + FLAME_STRIDE_PAD_BYTES / vb;
}
// The node-local step may address its arrays through buffer resources (32-bit offsets, range
// limit 2^32 - 1 bytes) only when every array it touches ends at least 16 bytes below 4 GiB, so
// that no access can meet the range limit whichever byte of it the hardware checks: the
// population arrays, and, when the launch reads forcing or writes a saved state
// (arith_arrays), the [n] arrays of the arithmetic type. Larger arrays take the 64-bit global
// addresses instead.
inline bool buffer_addressing_ok(const flame_params& p, bool arith_arrays) {
  const size_t limit = (size_t(1) << 32) - 16;
  const size_t n = static_cast<size_t>(p.nx) * p.ny * p.nz;
  const size_t arith = p.storage == FLAME_F64 ? 8 : 4;
  return population_stride(p) * value_bytes(p.storage) <= limit && (!arith_arrays || n * arith <= limit);
}
// Model bits of the step kernels: 1 = BGK fluid collision, 2 = electron MHD; 0 is the paper's.
inline int step_model(const flame_params& p) {
  return (p.collision == FLAME_COLLISION_BGK ? 1 : 0) | (p.magnetic == FLAME_MAGNETIC_EMHD ? 2 : 0);
}
inline bool mag_two_lattice(const flame_params& p) {
  return p.layout == FLAME_LAYOUT_AB || p.jmode == FLAME_J_STENCIL;
}
// Velocity sets: a run on anything but the paper's D3Q27 fluid and D3Q7 magnetic sets goes
// through the lattice-variant kernels (flame_lattice.hip).
inline bool lattice_variant(const flame_params& p) {
  return p.fluid_lattice != FLAME_FLUID_D3Q27 || p.magnetic_lattice != FLAME_MAGNETIC_D3Q7;
}
inline int fluid_count(const flame_params& p) { return p.fluid_lattice == FLAME_FLUID_D3Q19 ? 19 : 27; }
inline int mag_count(const flame_params& p) {
  return p.magnetic_lattice == FLAME_MAGNETIC_D3Q15 ? 15 : p.magnetic_lattice == FLAME_MAGNETIC_D3Q27 ? 27 : 7;
}
// Reverse mode and trace lattices are built for the paper's model and velocity sets only.
inline bool reverse_mode_built(const flame_params& p) { return step_model(p) == 0 && !lattice_variant(p); }
SetPtrs set_ptrs(const flame_ctx* c);

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2): hardware
// workgroup h runs on XCD h % 8. Remap so that XCD j processes one contiguous range of logical
// tiles (x fastest, then y, then z): neighbouring tiles, which share halo rows and the cache
// lines that shifted stores straddle, then sit behind the same L2.
#ifndef FLAME_XCD_REMAP
#define FLAME_XCD_REMAP 1
#endif
constexpr unsigned kXCDs = 8;

__device__ __forceinline__ void logical_block(unsigned gx, unsigned gy, unsigned gz, unsigned& bx, unsigned& by,
                                              unsigned& bz) {
  const unsigned total = gx * gy * gz;
  const unsigned h = blockIdx.x;
  unsigned l = h;
  if (FLAME_XCD_REMAP) {
    const unsigned q = total / kXCDs, r = total % kXCDs;
    const unsigned j = h % kXCDs, k = h / kXCDs;
    l = j * q + min(j, r) + k;
  }
  bx = l % gx;
  by = (l / gx) % gy;
  bz = l / (gx * gy);
}

// Threads of a row block of the node-local kernels: one row of nx nodes rounded up to whole
// wavefronts, at most 256 (longer rows take several blocks), so that short rows leave no wave
// of a block idle.
// Threads per row block of the node-local kernels, whose launch bounds are 256 threads: never more
// than that, whatever FLAME_ROW_THREADS asks for.
constexpr int kRowThreadsMax = 256;
inline unsigned row_threads(int nx) { return static_cast<unsigned>(std::min(kRowThreadsMax, (nx + 63) / 64 * 64)); }
inline unsigned row_threads(const flame_ctx* c) {
  return c->row_tx > 0 ? static_cast<unsigned>(std::min({c->row_tx, kRowThreadsMax, (c->p.nx + 63) / 64 * 64}))
                       : row_threads(c->p.nx);
}

// One fused step over the sets s, whose population arrays are stride elements apart; with
// save != null also writes the pre-collision state of every node (arithmetic type,
// [48 populations + 3 J][n]).
hipError_t launch_step(const flame_ctx* c, const SetPtrs& s, size_t stride, void* save);

// Lattice-variant kernels (flame_lattice.hip), each enqueued on the context's stream.
hipError_t variant_launch_step(const flame_ctx* c, const SetPtrs& s);
hipError_t variant_launch_init(const flame_ctx* c, const double* u, const double* b, const double* grad_u,
                               const double* grad_b);
hipError_t variant_launch_get(const flame_ctx* c, int deviations, double* dst);
hipError_t variant_launch_gather(const flame_ctx* c, int deviations, const int64_t* cells, int64_t cnt, double* out);
hipError_t variant_launch_set(const flame_ctx* c, int deviations, const double* src);
hipError_t variant_launch_moments(const flame_ctx* c, double* rho, double* u, double* b, double* j, double* divb);
hipError_t variant_launch_component(const flame_ctx* c, int field, int comp, double* out);
hipError_t variant_launch_reduce(const flame_ctx* c, double* partials);
// Rest populations of the lattice variants (host): f_rest[q], g_rest[3 m].
void variant_rest(const flame_params& p, double* f_rest, double* g_rest);

}  // namespace flame
