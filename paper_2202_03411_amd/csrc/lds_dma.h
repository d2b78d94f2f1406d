// Direct global -> LDS loads shared by the MFMA kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace msft {

// s_waitcnt immediates (gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt 6:4,
// lgkmcnt 11:8): wait until at most n vector-memory operations are outstanding
constexpr int waitcnt_vm(int n) { return (n & 15) | (7 << 4) | (15 << 8) | ((n >> 4) << 14); }

// One 16-byte piece per lane from global memory straight into LDS: lane l of the
// wave writes dst_wave + 16 l (dst_wave uniform over the wave).  Written as inline
// assembly so that the compiler does not wait for it before every read of the other
// ring slots (it cannot tell the slots apart); it produces no register result, and
// the caller waits for the memory counter before the barrier that publishes a slot.
// Vector-memory operations complete in issue order, so a wait the compiler places
// for its own loads only waits longer when such a piece is in flight.
// M0 is set inside the block; the compiler reserves M0 and uses it in none of the
// kernels that call this (their code has no other M0 access), so the clobber is
// declared for the reader only and its "reserved register" warning is silenced.
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
__device__ __forceinline__ void lds_dma16(const void* src, uint8_t* dst_wave)
{
    const uint32_t m0 = __builtin_amdgcn_readfirstlane(
        (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t*)dst_wave);
    asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
                 :
                 : "v"(src), "s"(m0)
                 : "memory", "m0");
}
// The same from a wave-uniform base (scalar registers) plus a 32-bit per-lane byte
// offset, so that no 64-bit address is formed per lane.
__device__ __forceinline__ void lds_dma16_s(const void* sbase, uint32_t voff, uint8_t* dst_wave)
{
    const uint32_t m0 = __builtin_amdgcn_readfirstlane(
        (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint8_t*)dst_wave);
    // (readfirstlane returns a signed int: widen through uint32_t, or a low word with
    // bit 31 set would be sign-extended into the high word)
    const uint64_t p = (uint64_t)(uintptr_t)sbase;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)p);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(p >> 32));
    const uint64_t base = ((uint64_t)hi << 32) | (uint64_t)lo;
    asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1"
                 :
                 : "v"(voff), "s"(base), "s"(m0)
                 : "memory", "m0");
}
#pragma clang diagnostic pop

}  // namespace msft
