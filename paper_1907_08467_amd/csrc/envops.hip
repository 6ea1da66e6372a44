// Env bookkeeping kernels: id validation and ROM tiling, eager reset from the
// reset cache, and small fills.
//
// Reset (paper, Section 3): at the end of an episode each env picks one of
// the cached initial states at random and copies it over its own state.  The
// pick is k = (R(seed, env, 2, episode) >> 32) mod K with the counter-based
// SplitMix64 draw R; the env keeps its id, ROM and step count, its episode
// count goes up by one, and its previous action becomes NOOP.
#include "vcs_device.h"

namespace vcs {

__global__ void k_fill_u32(uint32_t* p, uint32_t n, uint32_t v) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Start of a step or reset call: clear the per-call counters and, when the
// call validates ids, move its claim tag to the next value of its residue
// mod 16 (the up to 8 pipelines use residues 0-7, the scratch of the entry
// point that allocates nothing uses 8, so tags of different scratch sets
// never meet and each one only grows).  Kernels only (no memset), so a
// captured call replays correctly.
__global__ void k_step_begin(uint32_t* zero, uint32_t n_zero, uint32_t* tag, uint32_t residue) {
    for (uint32_t i = threadIdx.x; i < n_zero; i += blockDim.x) zero[i] = 0;
    if (tag && threadIdx.x == 0) *tag = ((*tag + 16u) & ~15u) | residue;
}

// Validate the ids of one call and count the valid ones per ROM.  An id out
// of range, or seen twice in the call, is marked invalid: its output gets
// done = 1 with the BAD_ID error and it is never dereferenced further.  An id
// is claimed by swapping the call's tag into claim[id]: a second position
// with the same id sees the tag already there.
__global__ void k_validate(const int32_t* ids, uint32_t n, uint32_t num_envs, const uint16_t* env_rom,
                           uint32_t* claim, const uint32_t* tag_ptr, uint32_t* counts, uint8_t* valid,
                           StepInfo* info, int32_t* reward, uint8_t* done, uint32_t* err_word) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t tag = *tag_ptr;
    const int32_t e = ids ? ids[i] : (int32_t)i;
    bool ok = e >= 0 && (uint32_t)e < num_envs;
    if (ok) ok = atomicExch(&claim[e], tag) != tag;
    valid[i] = ok ? 1 : 0;
    if (ok) {
        atomicAdd(&counts[env_rom[e]], 1u);
    } else {
        StepInfo si;
        si.k = 0; si.done = 1; si.err = (uint8_t)ERR_BAD_ID; si.slots = 0;
        if (info) info[i] = si;
        if (reward) reward[i] = 0;
        if (done) done[i] = 1;
        atomicOr(&err_word[0], ERR_BAD_ID);
        atomicMin(&err_word[1], e >= 0 ? (uint32_t)e : 0xFFFFFFFEu);
    }
}

// Tile offsets per ROM (one thread; the number of ROMs is small).  Tiles
// hold `width` envs (the last tile of a ROM fewer).
__global__ void k_tile_layout(const uint32_t* counts, uint32_t n_roms, uint32_t width, uint32_t* offsets,
                              uint32_t* fill, Tile* tiles, uint32_t* n_tiles) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint32_t t = 0;
    for (uint32_t r = 0; r < n_roms; ++r) {
        offsets[r] = t;
        fill[r] = 0;
        uint32_t c = counts[r];
        while (c > 0) {
            const uint32_t take = c > width ? width : c;
            tiles[t].rom = (int32_t)r;
            tiles[t].count = (int32_t)take;
            ++t;
            c -= take;
        }
    }
    *n_tiles = t;
}

__global__ void k_tile_fill(const int32_t* ids, uint32_t n, const uint16_t* env_rom, const uint8_t* valid,
                            uint32_t width, const uint32_t* offsets, uint32_t* fill, Tile* tiles) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !valid[i]) return;
    const int32_t e = ids ? ids[i] : (int32_t)i;
    const uint32_t r = env_rom[e];
    const uint32_t s = atomicAdd(&fill[r], 1u);
    Tile& T = tiles[offsets[r] + s / width];
    T.env[s % width] = e;
    T.out[s % width] = (int32_t)i;
}



// One workgroup (64 threads) per listed position.
__global__ void __launch_bounds__(64) k_reset(ResetArgs A) {
    const uint32_t i = blockIdx.x;
    if (i >= A.n) return;
    if (A.nfpo && threadIdx.x == 0) A.nfpo[i] = 0;    // set below for a reset env
    if (A.valid && !A.valid[i]) {
        if (A.obs)
            for (int j = threadIdx.x; j < kObsBytes / 16; j += blockDim.x)
                reinterpret_cast<uint4*>(A.obs + (size_t)i * kObsBytes)[j] = make_uint4(0, 0, 0, 0);
        return;
    }
    if (A.info) {
        const StepInfo si = A.info[i];
        if (!si.done || (si.err & ERR_BAD_ID)) return;
    }
    const int32_t e = A.ids ? A.ids[i] : (int32_t)i;
    if (e < 0 || (uint32_t)e >= A.num_envs) return;
    DevEnv* dst = &A.envs[e];
    const uint32_t rom = dst->rom_id, step = dst->step_idx, episode = dst->episode_idx;
    const uint64_t draw = rng_draw(rng_prefix(A.seed, (uint64_t)e, kResetPurpose), episode);
    const uint32_t k = (uint32_t)((draw >> 32) % A.K);
    const DevEnv* src = &A.cache_state[(size_t)rom * A.K + k];
    __syncthreads();   // every thread has read the env's bookkeeping before it is overwritten
    const uint4* s4 = reinterpret_cast<const uint4*>(src);
    uint4* d4 = reinterpret_cast<uint4*>(dst);
    if (threadIdx.x < sizeof(DevEnv) / 16) {
        uint4 q = s4[threadIdx.x];
        if (threadIdx.x == 12) {          // bytes 192..207: rom_id, step_idx, episode_idx
            q.x = rom;
            q.y = step;
            q.z = episode + 1;
        }
        if (threadIdx.x == 9) {           // bytes 144..159: prev_action (155) and err (156)
            q.z &= 0x00FFFFFFu;
            q.w &= 0xFFFFFF00u;
        }
        d4[threadIdx.x] = q;
    }
    if (A.nfpo) {       // no-ops after the copy: 2 + n frames to run, the obs comes from them
        if (threadIdx.x == 0) {
            const uint64_t d2 = rng_draw(rng_prefix(A.seed, (uint64_t)e, kNoopAfterPurpose), episode);
            A.nfpo[i] = (uint16_t)(2 + (d2 >> 32) % ((uint64_t)A.noop_max + 1));
        }
        return;
    }
    if (A.obs) {
        const uint4* os = reinterpret_cast<const uint4*>(A.cache_obs + ((size_t)rom * A.K + k) * kObsBytes);
        uint4* od = reinterpret_cast<uint4*>(A.obs + (size_t)i * kObsBytes);
        for (int j = threadIdx.x; j < kObsBytes / 16; j += blockDim.x) od[j] = os[j];
    }
}

void launch_reset(const ResetArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_reset, dim3(a.n), dim3(64), 0, s, a);
}
void launch_fill_u32(uint32_t* p, uint32_t n, uint32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
}
void launch_step_begin(uint32_t* zero, uint32_t n_zero, uint32_t* tag, uint32_t residue, hipStream_t s) {
    hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(256), 0, s, zero, n_zero, tag, residue);
}
void launch_validate(const int32_t* ids, uint32_t n, uint32_t num_envs, const uint16_t* env_rom,
                     uint32_t* claim, const uint32_t* tag, uint32_t* counts, uint8_t* valid, StepInfo* info,
                     int32_t* reward, uint8_t* done, uint32_t* err_word, hipStream_t s) {
    hipLaunchKernelGGL(k_validate, dim3((n + 255) / 256), dim3(256), 0, s, ids, n, num_envs, env_rom, claim,
                       tag, counts, valid, info, reward, done, err_word);
}
void launch_tile_layout(const uint32_t* counts, uint32_t n_roms, uint32_t width, uint32_t* offsets,
                        uint32_t* fill, Tile* tiles, uint32_t* n_tiles, hipStream_t s) {
    hipLaunchKernelGGL(k_tile_layout, dim3(1), dim3(64), 0, s, counts, n_roms, width, offsets, fill, tiles,
                       n_tiles);
}
void launch_tile_fill(const int32_t* ids, uint32_t n, const uint16_t* env_rom, const uint8_t* valid,
                      uint32_t width, const uint32_t* offsets, uint32_t* fill, Tile* tiles, hipStream_t s) {
    hipLaunchKernelGGL(k_tile_fill, dim3((n + 255) / 256), dim3(256), 0, s, ids, n, env_rom, valid, width,
                       offsets, fill, tiles);
}

}  // namespace vcs
