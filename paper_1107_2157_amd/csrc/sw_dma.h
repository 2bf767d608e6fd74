// LDS DMA helpers of the MFMA kernels (device code; included by .hip
// sources only).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

// LDS byte address of a __shared__ object.
__device__ __forceinline__ unsigned lds_addr(const void *p) {
    return (unsigned)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}

// One LDS DMA instruction (global_load_lds_dwordx4): lane l's 16 bytes at
// base + off (off in bytes, per lane) go to LDS byte address lds + 16 l
// (checked on MI355X with destinations below and above 64 KB).
// Asynchronous and counted in vmcnt like a load; written as asm so that the
// compiler, which does not see the LDS write, does not wait for it before
// every LDS read: the kernels wait for it themselves.
__device__ __forceinline__ void lds_dma16(const void *base, unsigned off, unsigned lds) {
    // (one wait state between the M0 write and its use by the DMA)
    asm volatile("s_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, %1" ::"v"(off), "s"(base), "s"(lds)
                 : "memory", "m0");
}

// Wait until at most n vector memory operations of this wave are
// outstanding (n wave-uniform; values above K wait for K).  Vector memory
// operations complete in issue order, so this leaves exactly the n newest
// in flight.
template <int K> __device__ __forceinline__ void wait_vm_upto(int n) {
    if constexpr (K > 0) {
        if (n >= K) {
            asm volatile("s_waitcnt vmcnt(%0)" ::"n"(K) : "memory");
            return;
        }
        wait_vm_upto<K - 1>(n);
    } else {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
}
