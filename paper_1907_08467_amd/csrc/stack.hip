// Frame stack: the last D observations of every env, resident in HBM.
//
// What it computes (paper, Section 5, "Memory limitations"): agents consume
// each env's last four 84x84 observations; the paper keeps them uncompressed
// and names compression as future work.  Here the ring of D observations per
// env lives in device memory, optionally packed to 4 bits per pixel (the
// gray level's top nibble, two pixels per byte).  A push after a step writes
// the step's observation into the env's ring -- into every slot when the
// env's episode ended (the new episode starts with D copies of its first
// observation) -- and writes the stacked observation [D][84][84], oldest
// first, each pixel the stored value widened back to 8 bits (identity for
// 8-bit storage, q * 17 for a 4-bit q).
#include "vcs_device.h"

namespace vcs {

struct StackArgs {
    uint8_t* ring;            // [num_envs][D][slot_bytes]
    uint8_t* head;            // [num_envs]: slot of the newest observation
    const int32_t* ids;       // NULL = position i is env i
    uint32_t n, num_envs, depth, bits;
    const uint8_t* obs;       // [n][84][84]
    const uint8_t* done;      // [n] or NULL
    uint8_t* out;             // [n][D][84][84] or NULL
};

constexpr uint32_t kObsWords = kObsBytes / 4;   // 1764 words of 4 pixels

// 4 pixels -> 4 nibbles (16 bits): pixel k's top nibble at bits 4k..4k+3
__device__ __forceinline__ uint32_t pack4(uint32_t w) {
    return ((w >> 4) & 0xF) | ((w >> 8) & 0xF0) | ((w >> 12) & 0xF00) | ((w >> 16) & 0xF000);
}
// 16 bits of nibbles -> 4 pixels, each q * 17
__device__ __forceinline__ uint32_t unpack4(uint32_t h) {
    const uint32_t w = (h & 0xF) | ((h & 0xF0) << 4) | ((h & 0xF00) << 8) | ((h & 0xF000) << 12);
    return w * 17u;   // 17 * q <= 255: no carry between bytes
}

// one workgroup (256 threads) per listed position
__global__ void __launch_bounds__(256) k_stack(StackArgs A) {
    const uint32_t i = blockIdx.x;
    if (i >= A.n) return;
    const int32_t e = A.ids ? A.ids[i] : (int32_t)i;
    if (e < 0 || (uint32_t)e >= A.num_envs) return;      // invalid ids are left alone
    const uint32_t D = A.depth;
    const uint32_t slot_words = A.bits == 4 ? kObsWords / 2 : kObsWords;
    uint32_t* ring = reinterpret_cast<uint32_t*>(A.ring) + (size_t)e * D * slot_words;
    const uint32_t* ob = reinterpret_cast<const uint32_t*>(A.obs + (size_t)i * kObsBytes);
    const bool fresh = A.done && A.done[i];
    const uint32_t old = A.head[e];
    const uint32_t h = fresh ? 0u : (old + 1 == D ? 0u : old + 1);
    __syncthreads();   // every thread has read the head before thread 0 moves it
    if (threadIdx.x == 0) A.head[e] = (uint8_t)h;
    // write the new observation (into every slot for a fresh episode)
    const uint32_t s0 = fresh ? 0 : h, s1 = fresh ? D : h + 1;
    if (A.bits == 4) {
        for (uint32_t j = threadIdx.x; j < kObsWords / 2; j += blockDim.x) {
            const uint32_t p = pack4(ob[2 * j]) | (pack4(ob[2 * j + 1]) << 16);
            for (uint32_t s = s0; s < s1; ++s) ring[s * slot_words + j] = p;
        }
    } else {
        for (uint32_t j = threadIdx.x; j < kObsWords; j += blockDim.x) {
            const uint32_t p = ob[j];
            for (uint32_t s = s0; s < s1; ++s) ring[s * slot_words + j] = p;
        }
    }
    if (!A.out) return;
    __syncthreads();   // the block's own ring writes are visible to its reads below
    uint32_t* out = reinterpret_cast<uint32_t*>(A.out + (size_t)i * D * kObsBytes);
    for (uint32_t d = 0; d < D; ++d) {
        uint32_t s = h + 1 + d;                // oldest first: the slot after the newest
        s = s >= D ? s - D : s;
        const uint32_t* src = ring + s * slot_words;
        uint32_t* dst = out + d * kObsWords;
        if (A.bits == 4) {
            for (uint32_t j = threadIdx.x; j < kObsWords / 2; j += blockDim.x) {
                const uint32_t p = src[j];
                dst[2 * j] = unpack4(p & 0xFFFF);
                dst[2 * j + 1] = unpack4(p >> 16);
            }
        } else {
            for (uint32_t j = threadIdx.x; j < kObsWords; j += blockDim.x) dst[j] = src[j];
        }
    }
}

void launch_stack(uint8_t* ring, uint8_t* head, const int32_t* ids, uint32_t n, uint32_t num_envs, uint32_t depth,
                  uint32_t bits, const uint8_t* obs, const uint8_t* done, uint8_t* out, hipStream_t s) {
    StackArgs a{ring, head, ids, n, num_envs, depth, bits, obs, done, out};
    hipLaunchKernelGGL(k_stack, dim3(n), dim3(256), 0, s, a);
}

}  // namespace vcs
