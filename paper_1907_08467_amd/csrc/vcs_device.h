// Device-side layouts shared by the vcs355 kernels and the host library.
//
// Env state lives in HBM as one 384-byte record per env (DevEnv).  A step
// loads a tile of 64 envs into one wave: RAM into LDS, CPU registers into
// VGPRs.  The interpreter writes, for each frame it renders, a row log: per
// scanline row a 32-byte snapshot of the render registers at the row's first
// visible pixel, and the register writes that land inside the row as 4-byte
// entries packed row after row into one stream, so the render kernel can
// draw every row and pixel independently and reads only the entries logged.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace vcs {

constexpr int kLanes = 64;             // envs per tile = one wave64
constexpr int kRows = 210;             // frame rows
constexpr int kCols = 160;             // frame columns
constexpr int kFirstRow = 34;          // frame row 0 = scanline 34 of the frame
constexpr int kObs = 84;
constexpr int kObsBytes = kObs * kObs;
constexpr int kFrameBytes = kRows * kCols;
// Row log of one frame: the 210 row snapshots, then the entry stream.
// Every emulated TIA write logs at most one entry.  The writes whose effect
// lands in one row's visible part (colour clocks 68..227 of a line) are made
// at 53 consecutive access cycles; all writes of an instruction happen at
// its last cycle, so the densest sequence is a BRK (3 pushes) at the first
// of those cycles, seven more 7-cycle BRKs and a 3-cycle store: 25 writes.
// A row also takes the frame-end entry, so a frame logs at most 210 * 25 + 1
// entries.
constexpr int kRowEntries = 25;        // max register writes inside one row's visible part
constexpr int kSnapBytes = 32;         // row snapshot: the render registers R[0..31]
constexpr int kSnapArea = 6784;        // 210 snapshots (6,720 B), padded to whole 128-byte lines
constexpr int kFrameEntries = 5280;    // entry stream capacity >= 210 * 25 + 1, in whole lines
constexpr int kFrameLogBytes = kSnapArea + 4 * kFrameEntries;   // 27,904
constexpr uint32_t kCountMask = 0x1F;  // snapshot byte 15: entries in the row (<= 26)
// snapshot bytes 28-29: index of the row's first entry in the stream (R[28..31]
// are no registers)
constexpr int kTiaRegs = 48;           // render registers + full-byte copies (R[0..47])
constexpr int kRomSlot = 32768;        // bytes per ROM slot (smaller ROMs use its start)

// TIA register file R[0..47] of an env, in snapshot order (TIA $06..$0F map
// to 0..9).  Bytes 0..31 are what a row snapshot records and a log entry's
// code names; 32..47 hold the last byte written to the registers the
// renderer sees only through the flag bits of R_FLAGS / R_FLAGS2.
enum : int {
    R_COLUP0 = 0, R_COLUP1, R_COLUPF, R_COLUBK, R_CTRLPF, R_REFP0, R_REFP1, R_PF0, R_PF1, R_PF2,
    R_GRP0 = 10, R_GRP1 = 11, R_P0X = 12, R_P1X = 13, R_VBLANK = 14,
    R_COUNT = 15,            // snapshot only: entries in the row, kRowOutside
    R_GRP0_OLD = 16, R_GRP1_OLD = 17, R_NUSIZ0 = 18, R_NUSIZ1 = 19, R_M0X = 20, R_M1X = 21, R_BLX = 22,
    R_FLAGS = 23,            // ENAM0 D1, ENAM1 D1, ENABL D1, ENABL (delayed) D1, VDELP0 D0, VDELP1 D0, VDELBL D0, RESMP0 D1
    R_FLAGS2 = 24,           // RESMP1 D1 in bit 0
    R_HMB = 25,              // 1 + the frame row whose pixels 0-7 an early HMOVE blanked (0 = none)
    // full bytes, in R_FLAGS bit order, then RESMP1 and the motion registers of missiles and ball
    R_ENAM0 = 32, R_ENAM1, R_ENABL, R_ENABL_OLD, R_VDELP0, R_VDELP1, R_VDELBL, R_RESMP0, R_RESMP1,
    R_HMM0 = 41, R_HMM1, R_HMBL,
    // entry-only codes
    R_END = 27,              // the frame ended: pixels from here on are outside
    R_RESMP = 0x30,          // + i: RESMPx; v0 = the new R_FLAGS (x = 0) / R_FLAGS2 (x = 1), v1 = missile x's position
    R_HMOVE = 0x40           // | BL motion nibble: HMOVE; v0 = P0 | P1 << 4, v1 = M0 | M1 << 4 motion nibbles
};
// snapshot byte 15: number of entries in the row, bit 7 = row outside the frame
constexpr uint32_t kRowOutside = 0x80;

// error bits (same values as the C header)
constexpr uint32_t ERR_ILLEGAL = 1, ERR_FRAME_CAP = 2, ERR_BAD_ACTION = 4, ERR_BAD_ID = 8, ERR_LOG = 16;

struct alignas(16) DevEnv {
    uint8_t ram[128];        //   0  RAM $80..$FF
    uint8_t tia[16];         // 128  render registers R[0..15]; [15] = 0
    uint8_t a, x, y, sp;     // 144
    uint8_t p, bank, vsync, hmp0;              // 148  bank: bank state bits 0-7
    uint8_t hmp1, tv, tshift, prev_action;     // 152  timer value / log2 interval
    uint8_t err, bank_hi;                      // 156  bank state bits 8-15
    uint16_t pc;                               // 158
    uint64_t cycle;          // 160  start cycle of the next instruction
    uint64_t frame_line0;    // 168  scanline of the write that began the frame
    int64_t tbase;           // 176  first cycle at which the last timer write is visible
    uint64_t instr;          // 184  instructions executed
    uint32_t rom_id, step_idx, episode_idx, pad1;   // 192
    uint8_t tia2[32];        // 208  R[16..47]
    uint16_t cx;             // 240  collision latches (bit 2r+1 / 2r = D7 / D6 of CX register r)
    uint8_t track_cx;        // 242  collision latches tracked
    uint8_t hmb_now;         // 243  an early HMOVE blanked pixels 0-7 of the line of `cycle`
    uint8_t reserved[12];    // 244
    uint8_t xram[128];       // 256  Superchip RAM
};
static_assert(sizeof(DevEnv) == 384, "DevEnv is 384 bytes");

// Cartridge mapping of one ROM.  The bank state of an env (16 bits) is a
// "virtual bank": the 4 KB bank of linear schemes (4K, F8, F6, F4 and their
// Superchip forms), the three E0 segment slices s0 | s1 << 3 | s2 << 6, or the
// 3F slice of the lower 2 KB.  The predecoded ROM holds 4096 words per
// virtual bank, so the instruction at (bank, pc) is one load for every scheme.
enum : uint32_t { CART_LINEAR = 0, CART_E0 = 1, CART_3F = 2 };
struct RomInfo {
    uint32_t kind;            // CART_*
    uint32_t hs_first;        // linear: first hotspot offset ($FF8 / $FF6 / $FF4)
    uint32_t hs_n;            // linear: number of banks when switched (0 = no hotspots)
    uint32_t sc;              // 1: Superchip RAM at $1000-$10FF
    uint32_t tf_last;         // 3F: ROM offset of the last 2 KB slice
    uint32_t tf_mask;         // 3F: slices - 1 (a power of two minus one)
    uint32_t n_vbanks;        // virtual banks (predecoded ROM = n_vbanks x 4096 words)
    uint32_t pre_off;         // this ROM's first word in the predecoded table
};

// ROM offset shown at cartridge address a (A12 set) under bank state `bank`
__host__ __device__ inline uint32_t cart_rom_off(uint32_t kind, uint32_t tf_last, uint32_t bank, uint32_t a) {
    const uint32_t lo = a & 0xFFF;
    if (kind == CART_LINEAR) return (bank << 12) | lo;
    if (kind == CART_E0) {
        const uint32_t seg = lo >> 10;
        const uint32_t sl = seg == 3 ? 7u : (bank >> (3 * seg)) & 7u;
        return (sl << 10) | (lo & 0x3FF);
    }
    return (lo < 0x800 ? (bank << 11) : tf_last) | (lo & 0x7FF);
}
__host__ __device__ inline uint32_t cart_rom_off(const RomInfo& R, uint32_t bank, uint32_t a) {
    return cart_rom_off(R.kind, R.tf_last, bank, a);
}

// Bank state after a data access to cartridge address a (hotspots)
__host__ __device__ inline uint32_t cart_hotspot(uint32_t kind, uint32_t hs_first, uint32_t hs_n, uint32_t bank,
                                                 uint32_t a) {
    const uint32_t lo = a & 0xFFF;
    if (kind == CART_LINEAR) {
        const uint32_t d = lo - hs_first;
        return d < hs_n ? d : bank;
    }
    if (kind == CART_E0 && lo - 0xFE0u < 24u) {
        const uint32_t sh = 3 * ((lo - 0xFE0) >> 3);
        return (bank & ~(7u << sh)) | ((lo & 7u) << sh);
    }
    return bank;
}

// The mapping packed into two words for the interpreter's scalar registers:
// a = kind | sc << 2 | hs_n << 4 | hs_first << 8, b = tf_last | tf_mask << 16
struct CartMap {
    uint32_t a, b;
};
__host__ __device__ inline CartMap pack_cart(const RomInfo& R) {
    return CartMap{R.kind | (R.sc << 2) | (R.hs_n << 4) | (R.hs_first << 8), R.tf_last | (R.tf_mask << 16)};
}

struct Tile {                 // up to 64 envs of one ROM, one per lane
    int32_t rom;
    int32_t count;            // envs in the tile (<= the launch's tile width)
    int32_t env[kLanes];      // env id per lane (-1 = idle lane)
    int32_t out[kLanes];      // output position per lane
};

struct StepInfo {             // per output position
    uint8_t k;                // frames emulated this step
    uint8_t done;
    uint8_t err;
    uint8_t slots;            // bit s: row-log slot s holds a complete frame
};

struct InterpArgs {
    const Tile* tiles;
    const uint32_t* n_tiles;  // device count of valid tiles (grid may be larger)
    DevEnv* envs;
    const uint8_t* roms;      // [n_roms][kRomSlot]
    const CartMap* cmap;      // [n_roms]
    const uint32_t* pre_off;  // [n_roms]: each ROM's first predecoded word
    const uint32_t* pre;      // predecoded ROMs (RomInfo::pre_off, n_vbanks)
    const uint8_t* actions;   // [n outputs]; NULL = NOOP
    const uint16_t* nframes_per_out;  // [n outputs] or NULL
    uint32_t nframes;         // frames per step when nframes_per_out is NULL
    uint32_t render_all;      // 1: log every frame (slot = f); 0: the last two (slot = f - (nfr - 2))
    uint32_t log_enabled;
    uint32_t early_stop;      // stop after the frame in which RAM[$D1] != 0
    uint32_t sticky_thr;
    uint32_t frameskip;       // for the sticky counter
    uint64_t seed;
    uint8_t* logs;            // [n outputs][n_slots][kFrameLogBytes]
    uint32_t n_slots;
    StepInfo* info;
    int32_t* reward;          // [n outputs] or NULL
    uint8_t* done;            // [n outputs] or NULL
    uint32_t* err_word;       // [0] bits, [1] smallest env id with an error
    unsigned long long* instr_total;   // [0] instructions (summed over lanes), [1] of them on the
                                       // scalar path, [2] wave instruction passes, [3] wave
                                       // scheduling rounds; or NULL
    uint32_t* queue;          // NULL: workgroup b runs tile b; else workgroups take
                              // tiles from this counter until it passes *n_tiles
    uint32_t track;           // collision latches tracked
    uint32_t count_step;      // 1: a step (the env's step counter advances); 0: the reset no-op
                              // frames of the envs whose frame count is not 0
    uint8_t* cx_logs;         // [n outputs][kFrameLogBytes]: logs of frames not rendered (track)
};

// SplitMix64 finaliser (Steele, Lea and Flood, OOPSLA 2014)
__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
// counter-based draw R(seed, id, purpose, n), split into a per-(env, purpose)
// prefix and the counter step
__host__ __device__ inline uint64_t rng_prefix(uint64_t seed, uint64_t id, uint64_t purpose) {
    return mix64(mix64(mix64(seed + kGamma) ^ id) ^ (purpose << 48));
}
__host__ __device__ inline uint64_t rng_draw(uint64_t prefix, uint64_t n) { return mix64(prefix ^ n); }
constexpr uint64_t kStickyPurpose = 1, kResetPurpose = 2, kNoopPurpose = 3, kNoopAfterPurpose = 4;

struct RenderArgs {
    const uint8_t* logs;      // [n][n_slots][kFrameLogBytes]
    uint32_t n_slots;
    const StepInfo* info;     // [n]
    uint8_t* frames;          // [n][n_slots][210][160] or NULL
    uint8_t* obs;             // [n][84][84] or NULL
    const uint8_t* gray;      // [128]
    uint32_t n;
    uint32_t force_obs;       // also for envs that ended (cache build)
    const uint16_t* only;     // NULL, or only positions with only[i] > 0 get an observation
};

struct ResetArgs {
    DevEnv* envs;
    const int32_t* ids;          // NULL = position i is env i
    uint32_t n;
    uint32_t num_envs;
    const StepInfo* info;        // NULL: reset every listed env; else only done ones
    const uint8_t* valid;        // NULL or per-position validity
    const DevEnv* cache_state;   // [n_roms][K]
    const uint8_t* cache_obs;    // [n_roms][K][84*84]
    uint32_t K;
    uint64_t seed;
    uint8_t* obs;                // [n][84][84] or NULL
    uint16_t* nfpo;              // NULL, or no-ops after the copy: [n] frames each position's
                                 // env must run next (2 + n drawn for a reset one, else 0);
                                 // the cache obs is then not copied
    uint32_t noop_max;
};

// host launchers (one per kernel)
// tile_envs: widest tile; rom_lds: bytes of ROM staged in LDS (8192), or 0 to
// read the cartridges from HBM
void launch_interp(const InterpArgs& a, uint32_t grid, uint32_t tile_envs, uint32_t rom_lds, hipStream_t s);
void launch_predecode(const uint8_t* rom, const RomInfo& info, uint32_t* pre, uint32_t track, hipStream_t s);
void launch_render_frames(const RenderArgs& a, uint32_t n_front_slots, uint32_t block, hipStream_t s);
void launch_render_obs(const RenderArgs& a, uint32_t block, hipStream_t s);
void launch_reset(const ResetArgs& a, hipStream_t s);
void launch_fill_u32(uint32_t* p, uint32_t n, uint32_t v, hipStream_t s);

// one layer of the policy network (layer = 0..4)
struct PolicyLayerArgs {
    const void* in;        // layer 0: u8 [n][4][84][84]; others: bf16 NHWC [n][H][H][Cin]
    const uint16_t* w;     // bf16 bits in operand order (policy_swizzle_index)
    const float* bias;     // [Npad]
    void* out;             // bf16 NHWC [n][OH][OH][N] (hidden) or f32 [n][32] (head)
    uint32_t M;            // n * OH * OH output positions, > 0
};
void launch_policy_layer(int layer, const PolicyLayerArgs& a, hipStream_t s);
// Where weight (channel c, reduction index k) of a layer with K = 32 KS
// reduction indices and NT 16-channel tiles goes in operand order: fragment
// (k-step k / 32, tile c / 16) is 64 lanes x 8 values, lane (c % 16) + 16 ((k % 32) / 8)
// holding values k % 8.
inline size_t policy_swizzle_index(uint32_t c, uint32_t k, uint32_t NT) {
    const uint32_t s = k / 32, j = c / 16, lane = (c % 16) + 16 * ((k % 32) / 8), t = k % 8;
    return (((size_t)s * NT + j) * 64 + lane) * 8 + t;
}
void launch_argmax(const float* logits, uint32_t n, uint8_t* actions, hipStream_t s);
void launch_stack(uint8_t* ring, uint8_t* head, const int32_t* ids, uint32_t n, uint32_t num_envs, uint32_t depth,
                  uint32_t bits, const uint8_t* obs, const uint8_t* done, uint8_t* out, hipStream_t s);
void launch_step_begin(uint32_t* zero, uint32_t n_zero, uint32_t* tag, uint32_t residue, hipStream_t s);
void launch_validate(const int32_t* ids, uint32_t n, uint32_t num_envs, const uint16_t* env_rom,
                     uint32_t* claim, const uint32_t* tag, uint32_t* counts, uint8_t* valid, StepInfo* info,
                     int32_t* reward, uint8_t* done, uint32_t* err_word, hipStream_t s);
void launch_tile_layout(const uint32_t* counts, uint32_t n_roms, uint32_t width, uint32_t* offsets,
                        uint32_t* fill, Tile* tiles, uint32_t* n_tiles, hipStream_t s);
void launch_tile_fill(const int32_t* ids, uint32_t n, const uint16_t* env_rom, const uint8_t* valid,
                      uint32_t width, const uint32_t* offsets, uint32_t* fill, Tile* tiles, hipStream_t s);

}  // namespace vcs
