// Device helpers shared by the kernels that keep per-frame state in a device
// workspace (streamed QC decoders, unrolled differentiable CBP).
#pragma once
#include "internal.hpp"

namespace cbp {

// A workgroup's workspace as a buffer resource (base and size in SGPRs):
// every state access is a buffer load/store with a 32-bit lane offset, so no
// 64-bit VGPR address is ever formed (and an offset past the end reads 0 /
// drops the store instead of faulting).
using u32x2 = __attribute__((ext_vector_type(2))) unsigned int;
using u32x4 = __attribute__((ext_vector_type(4))) unsigned int;
struct Ws {
    __amdgpu_buffer_rsrc_t r;
    __device__ float ld(uint32_t o) const {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)o, 0, 0));
    }
    __device__ void st(uint32_t o, float v) const {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)o, 0, 0);
    }
    __device__ float2 ld2(uint32_t o) const {
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)o, 0, 0);
        return make_float2(__uint_as_float(v.x), __uint_as_float(v.y));
    }
    __device__ void st2(uint32_t o, float2 v) const {
        const u32x2 u = {__float_as_uint(v.x), __float_as_uint(v.y)};
        __builtin_amdgcn_raw_buffer_store_b64(u, r, (int)o, 0, 0);
    }
    __device__ uint32_t ldb(uint32_t o) const { return __builtin_amdgcn_raw_buffer_load_b8(r, (int)o, 0, 0); }
    __device__ void stb(uint32_t o, bool v) const {
        __builtin_amdgcn_raw_buffer_store_b8((unsigned char)v, r, (int)o, 0, 0);
    }
    __device__ float4 ld4(uint32_t o) const {
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)o, 0, 0);
        return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z),
                           __uint_as_float(v.w));
    }
    __device__ void st4(uint32_t o, float4 v) const {
        const u32x4 u = {__float_as_uint(v.x), __float_as_uint(v.y), __float_as_uint(v.z),
                         __float_as_uint(v.w)};
        __builtin_amdgcn_raw_buffer_store_b128(u, r, (int)o, 0, 0);
    }
};
// raw buffer, 32-bit dword format (gfx9 family descriptor word 3)
constexpr int kBufferWord3 = 0x00020000;

struct Edge {
    int b, sh, ep, epsh, epr;
    bool last, first;
};
__device__ __forceinline__ Edge edge(const int4 *erec, int e) {
    const int *rec = reinterpret_cast<const int *>(erec) + 4 * (int64_t)e;
    const int x = ldc(rec, 0), w = ldc(rec, 3);
    return Edge{x & 0xffff, ldc(rec, 1), ldc(rec, 2), w & 0xffff, w >> 16, ((x >> 29) & 1) != 0,
                ((x >> 30) & 1) != 0};
}

}  // namespace cbp
