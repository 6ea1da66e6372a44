/*
 * CPU oracle for the batched Atari 2600 emulation path -- TEST INFRASTRUCTURE.
 *
 * A plain, slow, sequential emulator: one machine at a time, one CPU cycle
 * at a time, one pixel at a time.  It exists only to check the GPU library;
 * only the test suite, the smoke check and the CPU-baseline leg of the bench
 * may load it.  It shares no code, header or table with the GPU library.
 *
 * What it computes (paper, Section 3 "CUDA Learning Environment"): many
 * independent consoles, each a 6507 CPU + 128 B RAM + cartridge ROM + TIA
 * video, stepped with frameskip; frames rendered at 160x210; the observation
 * is the pixelwise maximum of the last two frames of each step; episodes
 * restart from a cache of 30 initial states built from 64 start-up frames
 * plus up to 30 random no-op frames.  The machine semantics the paper does
 * not spell out (6502 ISA, TIA/RIOT register map, timing conventions) follow
 * the public hardware definition and the conventions written next to each
 * function in machine.c and env.c.
 *
 * Machine-state record (384 bytes, little-endian), the exchange format that
 * both this oracle and the GPU library write independently:
 *    0 A   1 X   2 Y   3 SP   4 P   5 bank state bits 0-7   6..7 PC
 *    8..15  cycle      next instruction start cycle since power-on
 *   16..23  frame_line0   scanline of the write that began the current frame
 *   24 INTIM value a read at `cycle` would see   25 timer-expired flag (0/1)
 *   26..27 timer interval (1, 8, 64, 1024)
 *   28..29 timer phase: cycles since the last decrement (0 once expired)
 *   31 bank state bits 8-15
 *   32..159 RAM ($80..$FF)
 *  160 VSYNC 161 VBLANK 162 COLUP0 163 COLUP1 164 COLUPF 165 COLUBK
 *  166 CTRLPF 167 REFP0 168 REFP1 169 PF0 170 PF1 171 PF2 172 GRP0
 *  173 GRP1 174 HMP0 175 HMP1 176 P0 position 177 P1 position
 *  180..183 rom_id   184..187 step_idx   188..191 episode_idx
 *  192 prev_action   193 (0)   194 err bits   200..207 instructions executed
 *  208 NUSIZ0 209 NUSIZ1 210 ENAM0 211 ENAM1 212 ENABL 213 ENABL (delayed copy)
 *  214 GRP0 (delayed copy) 215 GRP1 (delayed copy) 216 VDELP0 217 VDELP1
 *  218 VDELBL 219 RESMP0 220 RESMP1 221 M0 position 222 M1 position
 *  223 ball position 224 HMM0 225 HMM1 226 HMBL
 *  227 1 when an early HMOVE blanked pixels 0-7 of the line of `cycle`
 *  228..229 collision latches (bit 2r+1 / 2r = D7 / D6 of CX register r)
 *  230 collision latches tracked (0/1)
 *  256..383 Superchip RAM (0 for other cartridges)
 *  all other bytes 0.
 *
 * Parity status: every function is pinned by the tests under tests/ (ISA
 * programs, exhaustive ADC/SBC tables, the datasheet cycle matrix, frame
 * invariants, render and preprocess special cases, SplitMix64 vectors),
 * except the palette-dependent gray values (project data, an input) and the
 * project conventions that have no outside reference (listed in the design
 * notes as readings of the paper).
 */
#ifndef VCS_ORACLE_H
#define VCS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_STATE_BYTES 384
#define ORC_FRAME_H 210
#define ORC_FRAME_W 160
#define ORC_OBS 84

enum { ORC_OK = 0, ORC_E_INVAL = -1, ORC_E_NOMEM = -2, ORC_E_ROM = -3, ORC_E_STATE = -5 };
enum { ORC_ERR_ILLEGAL = 1, ORC_ERR_FRAME_CAP = 2, ORC_ERR_BAD_ACTION = 4 };
enum { ORC_RENDER_ALL = 0, ORC_RENDER_LAST2 = 1 };

typedef struct {
    uint32_t num_envs;
    uint32_t frameskip;
    uint32_t sticky_threshold;   /* a frame repeats the previous action when
                                    (R >> 32) < threshold; 0 = off           */
    uint32_t reset_cache_k;      /* cached initial states per ROM (paper: 30) */
    uint32_t noop_max;           /* random no-op frames 0..noop_max (30)      */
    uint32_t startup_frames;     /* start-up frames (paper: 64)               */
    uint64_t seed;
    uint32_t render_mode;        /* ORC_RENDER_ALL or ORC_RENDER_LAST2        */
    uint32_t collisions;         /* 1: track the TIA collision latches        */
    uint32_t noop_after_copy;    /* 1: the random no-ops run after each reset's
                                    copy instead of being baked into the cache */
    uint8_t gray_lut[128];       /* gray value of colour index (c >> 1)       */
} oracle_config;

typedef struct oracle_ctx oracle_ctx;

int oracle_create(const oracle_config* cfg, oracle_ctx** out);
void oracle_destroy(oracle_ctx* ctx);
int oracle_set_threads(int n);
int oracle_get_threads(void);
int oracle_load_roms(oracle_ctx* ctx, uint32_t n_roms, const uint8_t* const* roms,
                     const uint32_t* rom_bytes, const uint32_t* schemes);
int oracle_assign(oracle_ctx* ctx, const uint16_t* env_rom);
int oracle_reset(oracle_ctx* ctx, const int32_t* env_ids, uint32_t n, uint8_t* obs);
int oracle_step(oracle_ctx* ctx, const int32_t* env_ids, const uint8_t* actions, uint32_t n,
                uint8_t* obs, int32_t* reward, uint8_t* done, uint8_t* frames, int render);
int oracle_get_state(oracle_ctx* ctx, uint32_t env, uint8_t* out);
int oracle_set_state(oracle_ctx* ctx, uint32_t env, const uint8_t* in);
int oracle_get_cache(oracle_ctx* ctx, uint32_t rom, uint32_t k, uint8_t* state, uint8_t* obs);
int oracle_poll_errors(oracle_ctx* ctx, uint32_t* first_env, uint32_t* bits);

/* bare-machine harness used by the ISA / device / render pins */
int oracle_power_on(const uint8_t* rom, uint32_t rom_bytes, uint32_t scheme, uint8_t* state);
int oracle_run_instructions(uint8_t* state, const uint8_t* rom, uint32_t rom_bytes,
                            uint32_t scheme, uint32_t n_instr, uint32_t action);
int oracle_batch_instructions(uint8_t* states, uint32_t n_states, const uint8_t* rom,
                              uint32_t rom_bytes, uint32_t scheme, uint32_t n_instr);
int oracle_run_frames(uint8_t* state, const uint8_t* rom, uint32_t rom_bytes, uint32_t scheme,
                      uint32_t n_frames, const uint8_t* actions, uint8_t* frames,
                      uint64_t* frame_end_cycle);
void oracle_preprocess(const uint8_t* f_prev, const uint8_t* f_last, const uint8_t* gray_lut,
                       uint8_t* obs);
uint64_t oracle_splitmix64_next(uint64_t* state);
uint64_t oracle_rng(uint64_t seed, uint64_t id, uint64_t purpose, uint64_t n);

#ifdef __cplusplus
}
#endif
#endif
