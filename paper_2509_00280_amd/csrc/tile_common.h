// Device helpers shared by the MTTKRP kernels.
#pragma once

#include "spt_internal.h"

namespace spt {

// Workgroups are dealt round-robin over the 8 XCDs.  Each XCD gets runs of
// kXcdChunk consecutive work indices (its L2 sees the key-order locality
// inside a run), and the runs of the 8 XCDs interleave over the whole index
// range, so a heavy stretch of the tensor is shared by all XCDs instead of
// landing on one (one contiguous eighth per XCD left the last XCD running
// 1.5x longer than the first on skewed tensors).  A bijection on [0, nwg):
// the indices past the last full round of 8 runs map to themselves.
constexpr int64_t kXcdChunk = 64;
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nwg) {
    const int64_t full = (nwg / (8 * kXcdChunk)) * (8 * kXcdChunk);
    if (b >= full) return b;
    const int64_t x = b & 7, j = b >> 3;
    return ((j / kXcdChunk) * 8 + x) * kXcdChunk + (j % kXcdChunk);
}

template <int VEC>
__device__ __forceinline__ void load_vec(const float *p, float (&x)[VEC]) {
    if constexpr (VEC == 4) {
        const float4 t = *reinterpret_cast<const float4 *>(p);
        x[0] = t.x;
        x[1] = t.y;
        x[2] = t.z;
        x[3] = t.w;
    } else {
#pragma unroll
        for (int q = 0; q < VEC; ++q) x[q] = p[q];
    }
}

// A factor matrix seen as a structured buffer whose records are its rows
// (stride R floats): a gather passes the row index and the column's byte
// offset straight to the load, with no address arithmetic, and rows past
// `rows` read as zero.  The descriptor is wave-uniform (SGPRs); R <= 4095.
typedef int spt_i4 __attribute__((ext_vector_type(4)));
typedef float spt_f4 __attribute__((ext_vector_type(4)));
typedef uint32_t spt_u2 __attribute__((ext_vector_type(2)));
typedef uint32_t spt_u4 __attribute__((ext_vector_type(4)));
__device__ spt_f4 spt_row_load4(spt_i4 rsrc, int vindex, int voffset, int soffset, int aux) __asm(
    "llvm.amdgcn.struct.buffer.load.v4f32");
__device__ float spt_row_load1(spt_i4 rsrc, int vindex, int voffset, int soffset, int aux) __asm(
    "llvm.amdgcn.struct.buffer.load.f32");

__device__ __forceinline__ spt_i4 row_rsrc(const float *base, int R, uint32_t rows) {
    const uint64_t p = (uint64_t)base;
    spt_i4 r;
    r.x = (int)(uint32_t)p;
    r.y = (int)(((uint32_t)(p >> 32) & 0xFFFFu) | ((uint32_t)(R * 4) << 16));  // base[47:32] | stride
    r.z = (int)rows;                                                            // records
    r.w = 0x00020000;                                                           // 32-bit data format
    return r;
}

template <int VEC>
__device__ __forceinline__ void load_row_vec(spt_i4 rsrc, uint32_t row, int col, float (&x)[VEC]) {
    if constexpr (VEC == 4) {
        const spt_f4 t = spt_row_load4(rsrc, (int)row, col * 4, 0, 0);
        x[0] = t.x;
        x[1] = t.y;
        x[2] = t.z;
        x[3] = t.w;
    } else {
#pragma unroll
        for (int q = 0; q < VEC; ++q) x[q] = spt_row_load1(rsrc, (int)row, (col + q) * 4, 0, 0);
    }
}

// The codec held in VGPRs: lane l of every wave keeps run descriptors l,
// l + 64 and l + 128 and the run bound rb[l / 5][l % 5].  Decoding reads them
// with v_readlane at wave-uniform indices: no memory access, no LDS wait.
struct CodecRegs {
    uint32_t r0, r1, r2, rb;
};

__device__ __forceinline__ CodecRegs load_codec_regs(const Codec &c) {
    const int lane = threadIdx.x & 63;
    CodecRegs cr;
    cr.r0 = lane < c.nruns ? c.run[lane] : 0u;
    cr.r1 = lane + 64 < c.nruns ? c.run[lane + 64] : 0u;
    cr.r2 = lane + 128 < c.nruns ? c.run[lane + 128] : 0u;
    cr.rb = lane < kMaxModes * 5 ? (uint32_t)(&c.rb[0][0])[lane] : 0u;
    return cr;
}

__device__ __forceinline__ uint32_t run_desc(const CodecRegs &cr, int r) {
    if (r < 64) return __builtin_amdgcn_readlane(cr.r0, r);
    if (r < 128) return __builtin_amdgcn_readlane(cr.r1, r - 64);
    return __builtin_amdgcn_readlane(cr.r2, r - 128);
}

// Coordinate of mode k from the four 32-bit words of one key.  A descriptor
// d packs word | kpos << 8 | cpos << 16 | len << 24 (len <= 31).
__device__ __forceinline__ uint32_t decode_mode(const CodecRegs &cr, int k, int nwords, const uint32_t (&w)[4]) {
    uint32_t x = 0;
#pragma unroll
    for (int word = 0; word < 4; ++word) {
        if (word < nwords) {
            const int r0 = __builtin_amdgcn_readlane(cr.rb, k * 5 + word);
            const int r1 = __builtin_amdgcn_readlane(cr.rb, k * 5 + word + 1);
            for (int r = r0; r < r1; ++r) {
                const uint32_t d = run_desc(cr, r);
                x |= __builtin_amdgcn_ubfe(w[word], (d >> 8) & 31u, d >> 24) << ((d >> 16) & 31u);
            }
        }
    }
    return x;
}

// In-place exclusive scan of n u32 values in LDS by a block of nthreads
// (n a multiple of nthreads); wsum holds one entry per wave.
__device__ __forceinline__ void block_scan_lds(uint32_t *a, int n, int nthreads, uint32_t *wsum) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per = n / nthreads;
    uint32_t *p = a + tid * per;
    uint32_t local = 0;
    for (int i = 0; i < per; ++i) local += p[i];
    uint32_t x = local;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint32_t run = x - local;
    for (int w = 0; w < wave; ++w) run += wsum[w];
    for (int i = 0; i < per; ++i) {
        const uint32_t v = p[i];
        p[i] = run;
        run += v;
    }
    __syncthreads();
}

__device__ __forceinline__ uint32_t mix_hash(uint32_t r) {
    r ^= r >> 16;
    r *= 0x7feb352dU;
    r ^= r >> 15;
    return r;
}

}  // namespace spt
