// Host-side context and launcher declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <string>

#include "../../include/flame.h"
#include "flame_device.h"

struct flame_ctx {
  flame_params p{};
  int device = 0;
  hipStream_t stream = nullptr;
  size_t n = 0;              // nodes
  void* storage = nullptr;   // caller-owned populations
  int parity = 0;            // AA in-place sets: 0 = canonical slots, 1 = swapped slots
  int cur = 0;               // two-lattice sets: index of the copy holding the current state
  int64_t steps = 0;
  double frest[27]{};        // f^mhd(0)(1, 0, b0)
  double omega = 0, omega_b = 0;
  double cfl = 0;
  std::string err;
  // library-owned scratch
  double* red_partials = nullptr;
  int red_blocks = 0;
  double* spec_real = nullptr;
  void* spec_cplx = nullptr;
  double* spec_partials = nullptr;
  int spec_blocks = 0;
  int spec_nshells = 0;
  hipfftHandle plan{};
  bool plan_ok = false;
};

namespace flame {

// Pointers to the population sets of the current step.
struct SetPtrs {
  void* f_src;
  void* f_dst;
  void* g_src;
  void* g_dst;
  bool fluid_aa;     // fluid set updated in place
  bool mag_aa;       // magnetic set updated in place
};

inline size_t value_bytes(int storage) { return storage == FLAME_F64 ? 8 : storage == FLAME_F32 ? 4 : 2; }
inline bool mag_two_lattice(const flame_params& p) {
  return p.layout == FLAME_LAYOUT_AB || p.jmode == FLAME_J_STENCIL;
}
SetPtrs set_ptrs(const flame_ctx* c);

hipError_t launch_step(const flame_ctx* c, const SetPtrs& s);

}  // namespace flame
