// Array access of the step and adjoint kernels: 32-bit node offsets from wave-uniform array
// bases, by 64-bit global addresses or by buffer resources.
#ifndef FLAME_ACCESS_H
#define FLAME_ACCESS_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "flame_device.h"

namespace flame {

#ifndef FLAME_NT_STORES
#define FLAME_NT_STORES 1
#endif

// Addresses: every array is indexed from a wave-uniform base (set + q * n, held in scalar
// registers) by a 32-bit per-lane node offset. A thread's nine in-plane neighbour offsets
// (x + dx, y + dy) are loop invariants; the plane offset z * nx * ny is uniform. The library
// limits each array to 4 GiB so byte offsets fit in 32 bits.
struct Rows {
  uint32_t r[3][3];   // [dx + 1][dy + 1] -> wrap(y + dy) * nx + wrap(x + dx)
  __device__ __forceinline__ Rows(int x, int y, int nx, int ny) {
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
        r[dx + 1][dy + 1] = static_cast<uint32_t>(wrap(y + dy, ny)) * nx + static_cast<uint32_t>(wrap(x + dx, nx));
  }
  __device__ __forceinline__ uint32_t at(int dx, int dy) const { return r[dx + 1][dy + 1]; }
};

// Addressing of the arrays. Every array spans at most 4 GiB (checked by the entry points), so an
// access is a wave-uniform array base plus a 32-bit per-lane byte offset. Global:
// 64-bit flat-global addresses formed per access in vector registers. Buffer: a buffer resource
// per array (base in scalar registers, no range limit below 4 GiB, raw addressing) and the 32-bit
// offset as the only per-lane operand, which takes the 64-bit address arithmetic off the vector
// ALU (about 140 of the node-local step's 1240 vector instructions per node at FP16 storage).
// Non-temporal stores unless FLAME_NT_STORES is 0.
enum class Addr { Global, Buffer };
typedef unsigned int U32x2 __attribute__((ext_vector_type(2)));
template <typename S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const S* base) {
  // stride 0, num_records 2^32 - 1, dword 3 of a raw 32-bit-format buffer on gfx9
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<S*>(base), 0, 0xFFFFFFFF, 0x00020000);
}
template <Addr A, typename S>
__device__ __forceinline__ S ld(const S* base, uint32_t off) {
  const uint32_t vo = off * static_cast<uint32_t>(sizeof(S));
  if constexpr (A == Addr::Buffer) {
    if constexpr (sizeof(S) == 2)
      return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b16(rsrc_of(base), vo, 0, 0));
    else if constexpr (sizeof(S) == 4)
      return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(rsrc_of(base), vo, 0, 0));
    else
      return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(rsrc_of(base), vo, 0, 0));
  } else {
    return *reinterpret_cast<const S*>(reinterpret_cast<const char*>(base) + vo);
  }
}
template <Addr A, typename S>
__device__ __forceinline__ void st(S* base, uint32_t off, S v) {
  const uint32_t vo = off * static_cast<uint32_t>(sizeof(S));
  if constexpr (A == Addr::Buffer) {
    constexpr int aux = FLAME_NT_STORES ? 2 : 0;   // 2: the non-temporal hint
    if constexpr (sizeof(S) == 2)
      __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(short, v), rsrc_of(base), vo, 0, aux);
    else if constexpr (sizeof(S) == 4)
      __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), rsrc_of(base), vo, 0, aux);
    else
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U32x2, v), rsrc_of(base), vo, 0, aux);
  } else {
    S* p = reinterpret_cast<S*>(reinterpret_cast<char*>(base) + vo);
    if (FLAME_NT_STORES)
      __builtin_nontemporal_store(v, p);
    else
      *p = v;
  }
}

// Plane offsets of z - 1, z, z + 1 (periodic), uniform across the workgroup.
struct Planes {
  uint32_t p[3];
  __device__ __forceinline__ Planes(int z, int nz, uint32_t plane) {
    p[0] = static_cast<uint32_t>(wrap(z - 1, nz)) * plane;
    p[1] = static_cast<uint32_t>(z) * plane;
    p[2] = static_cast<uint32_t>(wrap(z + 1, nz)) * plane;
  }
  __device__ __forceinline__ uint32_t at(int dz) const { return p[dz + 1]; }
};

// Buffer addressing is used when every array the kernel touches ends at least 16 bytes below
// 4 GiB, so that no access can meet the range limit whichever byte of it the hardware checks.
inline bool buffer_fits(size_t array_bytes) { return array_bytes <= (size_t(1) << 32) - 16; }

}  // namespace flame

#endif
