/*
 * vcs355 -- batched Atari 2600 emulation on one MI355X (gfx950), C ABI.
 *
 * The operation (paper, Section 3 "CUDA Learning Environment" and the
 * footnote on raw frames in Section 1): many independent consoles (6507 CPU,
 * 128 B RAM, cartridge ROM, TIA video, RIOT timer) step in lockstep on the
 * GPU; an env step emulates `frameskip` frames; frames are 160x210; the
 * observation is the pixelwise maximum of the last two frames of the step,
 * downsampled to 84x84 gray; episodes restart from a per-ROM cache of 30
 * initial states built from 64 start-up frames and up to 30 random no-op
 * frames.  Observations stay in device memory.
 *
 * Machine semantics the paper leaves open (6502 ISA, TIA/RIOT maps, timing,
 * frame boundary, palette, preprocessing arithmetic, sticky actions) follow
 * the conventions stated with each kernel in the library sources; they are
 * the same conventions the test oracle implements independently.
 *
 * Conventions for every call:
 *  - "_dev" pointers are device pointers on the context's device, owned by
 *    the caller; "_host" pointers are host memory, read (or written) before
 *    the call returns.
 *  - `stream` is a hipStream_t (NULL = the default stream).  vcs_reset and
 *    vcs_step only enqueue work on it and never synchronise.
 *  - Return values: VCS_OK or a negative VCS_E_* code; the message of the
 *    last failure on the calling thread is in vcs_last_error().
 *  - Argument errors the host can see (NULL pointers, n > max_batch, bad
 *    sizes) are rejected before anything is enqueued.  Errors only the device
 *    can see (an env id out of range or repeated in one call, an action >= 18,
 *    an undocumented opcode, a frame that never ends) set per-env error bits
 *    that vcs_poll_errors reports; such envs report done = 1 and restart from
 *    the cache; out-of-range ids are skipped, never dereferenced.
 *  - One context must not be used from two threads at once.
 */
#ifndef VCS355_H
#define VCS355_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VCS_STATE_BYTES 384      /* machine-state record, see vcs_get_state */
#define VCS_FRAME_H 210
#define VCS_FRAME_W 160
#define VCS_OBS 84
#define VCS_N_ACTIONS 18

enum {
    VCS_OK = 0,
    VCS_E_INVAL = -1,   /* bad argument */
    VCS_E_NOMEM = -2,   /* device or host allocation failed */
    VCS_E_ROM = -3,     /* ROM size / bank scheme not supported */
    VCS_E_HIP = -4,     /* a HIP runtime call failed */
    VCS_E_STATE = -5,   /* call out of order (e.g. step before assign) */
    VCS_E_BUDGET = -6   /* the allocation would exceed hbm_budget_bytes */
};

/* cartridge schemes (vcs_load_roms) */
enum {
    VCS_BANK_4K = 0,     /* 2 or 4 KB, no banks (2 KB shows twice) */
    VCS_BANK_F8 = 1,     /* 8 KB: 2 x 4 KB banks, hotspots $1FF8-$1FF9 */
    VCS_BANK_F6 = 2,     /* 16 KB: 4 banks, hotspots $1FF6-$1FF9 */
    VCS_BANK_F4 = 3,     /* 32 KB: 8 banks, hotspots $1FF4-$1FFB */
    VCS_BANK_F8SC = 4,   /* F8/F6/F4 with the Superchip's 128 B of RAM: */
    VCS_BANK_F6SC = 5,   /*   written at $1000-$107F, read at $1080-$10FF */
    VCS_BANK_F4SC = 6,
    VCS_BANK_E0 = 7,     /* 8 KB: 8 x 1 KB slices; $1C00-$1FFF fixed to slice 7,
                            segment k (0-2) set to slice n by an access to $1FE0 + 8k + n */
    VCS_BANK_3F = 8      /* 4, 8, 16 or 32 KB of 2 KB slices; $1800-$1FFF fixed to the
                            last one, $1000-$17FF set to slice v mod S by writing v to $00-$3F */
};
enum { VCS_RENDER_ALL = 0, VCS_RENDER_LAST2 = 1 };

/* per-env error bits (vcs_poll_errors) */
enum {
    VCS_ERR_ILLEGAL = 1,      /* undocumented opcode executed */
    VCS_ERR_FRAME_CAP = 2,    /* no VSYNC within 320 scanlines */
    VCS_ERR_BAD_ACTION = 4,   /* action >= 18 */
    VCS_ERR_BAD_ID = 8,       /* env id out of range or repeated in one call */
    VCS_ERR_LOG = 16          /* render log row capacity exceeded */
};

typedef struct {
    uint32_t num_envs;          /* resident envs */
    uint32_t frameskip;         /* frames per step: 1..255, and at most 8 with
                                   VCS_RENDER_ALL (every frame of a step gets a
                                   frame slot; a step records which slots it
                                   completed in 8 bits); VCS_E_INVAL otherwise.
                                   The paper counts 4 emulated frames per
                                   training frame (Section 1, the footnote on
                                   raw frames). */
    uint32_t sticky_threshold;  /* a frame repeats the previous frame's action
                                   when (R(seed, env, 1, step*frameskip+f) >> 32)
                                   < threshold; floor(p * 2^32); 0 = off   */
    uint32_t reset_cache_k;     /* cached initial states per ROM (paper: 30) */
    uint32_t noop_max;          /* no-op frames per cache entry: 0..noop_max (30) */
    uint32_t startup_frames;    /* start-up frames per cache entry (paper: 64)   */
    uint64_t seed;              /* seed of the counter-based RNG (SplitMix64)    */
    uint32_t render_mode;       /* VCS_RENDER_ALL: every frame is rendered;
                                   VCS_RENDER_LAST2: only frames frameskip-2 and
                                   frameskip-1 of a step (the two the
                                   observation needs)                           */
    uint32_t max_batch;         /* largest n of one step/reset call (0 = num_envs) */
    uint64_t hbm_budget_bytes;  /* cap on device memory the context allocates; 0 = none */
    int32_t device;             /* HIP device ordinal */
    uint32_t pipelines;         /* step pipelines (0 = 1, at most 8): each has its own
                                   scratch of max_batch envs, so calls on different
                                   pipelines may run concurrently (vcs_step_pipe) */
    uint32_t collisions;        /* 1: track the TIA collision latches (CXM0P..CXPPMM
                                   read what the frame's pixels so far set, CXCLR
                                   clears them; every frame is then logged and scanned,
                                   at some cost); 0: they read 0 */
    uint32_t noop_after_copy;   /* 0: the random no-op frames are baked into the
                                   reset-cache entries (paper, Section 3: the cache
                                   removes the per-reset frames); 1: the other
                                   reading: the entries stop two frames before the
                                   end of the start-up and every reset (assign,
                                   vcs_reset, eager) runs 2 + n NOOP frames with
                                   n = (R(seed, env, 4, episode) >> 32) mod
                                   (noop_max + 1), no sticky draw, the step counter
                                   unchanged; the reset's observation comes from the
                                   last two of them.  Needs startup_frames >= 2. */
    uint8_t gray_lut[128];      /* gray level of colour index (colour >> 1)      */
} vcs_config;

typedef struct vcs_ctx vcs_ctx;

/* Create a context: validates the config, allocates env state, render logs
   and scratch on `device`.  VCS_E_BUDGET when they exceed the budget. */
int vcs_create(const vcs_config* cfg, vcs_ctx** out);
void vcs_destroy(vcs_ctx* ctx);

/* The cartridges the consoles run (paper, Section 3: the first kernel reads
   the ROM instructions of each emulated console; the emulator runs the
   console, not game-specific code, so any cartridge loads).
   Copy n_roms cartridges to the device.  rom_bytes[r] must be a size the
   scheme takes (see VCS_BANK_*; VCS_E_ROM otherwise).  Bank hotspots switch
   on any data access, before it; instruction fetches see ROM even in the
   Superchip RAM window, and a read of its write port returns 0.  Power-on
   bank: the last 4 KB bank (F8/F6/F4), E0 slices 4, 5, 6, 3F slice 0.  The
   host buffers are copied; the caller keeps ownership. */
int vcs_load_roms(vcs_ctx* ctx, uint32_t n_roms, const uint8_t* const* rom_host,
                  const uint32_t* rom_bytes, const uint32_t* scheme);

/* The reset cache (paper, Section 3: instead of emulating the start of every
   episode, an env that ends restarts from one of a set of cached initial
   states, each made by 64 start-up frames and a random number of no-op
   frames, up to 30; 30 states per game).
   env_rom_host[num_envs]: the ROM of every env.  Builds each ROM's reset cache
   on the device (power-on, run to the first frame end, startup_frames NOOP
   frames, n_k NOOP frames; with noop_after_copy: startup_frames - 2 frames
   and no no-ops) and puts every env into a cache state (as vcs_reset, its
   no-op frames included).  Synchronises the device. */
int vcs_assign(vcs_ctx* ctx, const uint16_t* env_rom_host);

/* The environment's reset (paper, Section 3: a reset copies one of the
   cached initial states, chosen at random, into the env).
   Restart envs env_ids_dev[0..n) (NULL = envs 0..n-1) from a random cache
   entry (with noop_after_copy, then their 2 + n NOOP frames);
   obs_dev[n][84][84] (may be NULL) receives their observations: the cache
   entry's, or with noop_after_copy the one made from the last two of those
   frames.  Listed ids out of range or repeated are skipped (obs 0) and set
   VCS_ERR_BAD_ID. */
int vcs_reset(vcs_ctx* ctx, const int32_t* env_ids_dev, uint32_t n, uint8_t* obs_dev, void* stream);

/* The environment's step (paper, Section 1: environments execute a set of
   actions and produce observable states and rewards; its footnote on raw
   frames: every emulated frame counts, one in four becomes training input;
   Section 3: the input of the learner is the pixelwise maximum of the last
   two frames of four, frames are rendered in GPU memory, and an env whose
   episode ended restarts from a cached initial state).
   One env step for envs env_ids_dev[0..n) (NULL = envs 0..n-1) with
   actions_dev[n] in [0, 18).  Outputs, indexed like env_ids_dev:
     obs_dev[n][84][84]    observation (for envs that ended: the cache entry's,
                           or with noop_after_copy the one after their no-ops)
     reward_dev[n]         change of the BCD score byte at $D0 over the step
     done_dev[n]           1 when RAM[$D1] became non-zero (or the env faulted);
                           the env is then already restarted from the cache
                           (its no-op frames run, with noop_after_copy)
     frames_dev            NULL, or [n][F][210][160] palette-index frames with
                           F = frameskip (RENDER_ALL) or 2 (RENDER_LAST2, the
                           frames frameskip-2 and frameskip-1); frames that
                           were not emulated (the step stopped early) are 0. */
int vcs_step(vcs_ctx* ctx, const int32_t* env_ids_dev, const uint8_t* actions_dev, uint32_t n,
             uint8_t* obs_dev, int32_t* reward_dev, uint8_t* done_dev, uint8_t* frames_dev,
             void* stream);

/* vcs_step on pipeline `pipe` (vcs_step uses pipeline 0).  Calls on different
   pipelines may be in flight at once, on different streams, provided they
   list disjoint env ids: each env's steps then happen in the order the calls
   were made for it, and its results are those it would get from the same
   calls made one at a time.  VCS_E_INVAL for pipe >= pipelines. */
int vcs_step_pipe(vcs_ctx* ctx, uint32_t pipe, const int32_t* env_ids_dev, const uint8_t* actions_dev, uint32_t n,
                  uint8_t* obs_dev, int32_t* reward_dev, uint8_t* done_dev, uint8_t* frames_dev, void* stream);

/* vcs_step for callers that cannot allocate device memory (code under HIP
   graph capture, tight serving loops, harnesses that forbid hipMalloc): no
   device or host allocation, no event, no synchronisation.  Its scratch (row
   logs of the last two frames of each env, collision logs, step info, id
   validity, tiles, counters) is a static device array of 43.7 MB that every
   GPU the library runs on holds until the process ends, shared by every call
   and context on that GPU: calls on one GPU that overlap in time (different
   streams, or different host threads) race and must be serialised by the
   caller.  Limits: n <= 512 envs per call, at most 1024 ROMs loaded, and a
   context without noop_after_copy (VCS_E_INVAL otherwise).  Arguments and
   results as vcs_step, without the frames output: observations, rewards,
   done flags and env states equal those of vcs_step on the same inputs. */
int vcs_step_noalloc(vcs_ctx* ctx, const int32_t* env_ids_dev, const uint8_t* actions_dev, uint32_t n,
                     uint8_t* obs_dev, int32_t* reward_dev, uint8_t* done_dev, void* stream);

/* Machine-state record (384 bytes, little-endian) of one env:
     0 A  1 X  2 Y  3 SP  4 P  5 bank state bits 0-7  6..7 PC
     8..15 cycle (start of the next instruction, since power-on)
    16..23 scanline of the write that began the current frame
    24 INTIM a read at `cycle` would return   25 timer expired (0/1)
    26..27 timer interval (1, 8, 64, 1024)   28..29 cycles since the last
           decrement (0 once expired)   31 bank state bits 8-15 (the state:
           the 4 KB bank; E0 slices s0 | s1 << 3 | s2 << 6; 3F the lower slice)
    32..159 RAM $80..$FF
   160 VSYNC 161 VBLANK 162 COLUP0 163 COLUP1 164 COLUPF 165 COLUBK 166 CTRLPF
   167 REFP0 168 REFP1 169 PF0 170 PF1 171 PF2 172 GRP0 173 GRP1 174 HMP0
   175 HMP1 176 P0 position 177 P1 position
   180..183 rom_id 184..187 step count 188..191 episode count 192 previous
   action 194 error bits 200..207 instructions executed
   208 NUSIZ0 209 NUSIZ1 210 ENAM0 211 ENAM1 212 ENABL 213 ENABL (delayed copy)
   214 GRP0 (delayed copy) 215 GRP1 (delayed copy) 216 VDELP0 217 VDELP1
   218 VDELBL 219 RESMP0 220 RESMP1 221 M0 position 222 M1 position
   223 ball position 224 HMM0 225 HMM1 226 HMBL 227 1 when an early HMOVE
   blanked pixels 0-7 of the line of `cycle` 228..229 collision latches (bit
   2r+1 / 2r = D7 / D6 of CX register r) 230 latches tracked (vcs_config
   .collisions; set_state takes the context's)
   256..383 Superchip RAM; other bytes 0.
   get/set synchronise the device. */
int vcs_get_state(vcs_ctx* ctx, uint32_t env_id, uint8_t* out_host);
int vcs_set_state(vcs_ctx* ctx, uint32_t env_id, const uint8_t* in_host);

/* Cache entry k of ROM `rom`: state record and 84x84 observation (host). */
int vcs_get_cache(vcs_ctx* ctx, uint32_t rom, uint32_t k, uint8_t* state_host, uint8_t* obs_host);

/* Error bits OR-ed over all envs since the last poll, and the smallest env id
   that raised one (0xFFFFFFFF if none); clears them.  Synchronises. */
int vcs_poll_errors(vcs_ctx* ctx, uint32_t* first_env, uint32_t* bits);

/* Instructions emulated by the last vcs_step (sum over its envs); synchronises.
   Used to report emulated-instruction throughput. */
int vcs_last_step_instructions(vcs_ctx* ctx, uint64_t* out);

/* out2[0]: instructions emulated by the last vcs_step; out2[1]: how many of
   them ran in wave-uniform mode (every lane of a wave at the same PC, bank
   and cycle, so fetch, decode and timing ran once for the wave).
   Synchronises. */
int vcs_last_step_stats(vcs_ctx* ctx, uint64_t* out2);

/* Divergence of the last vcs_step (paper, Section 4: threads of one warp
   that take different branches run their paths one after another, and full
   divergence would leave one thread of 32 busy).  out4[0]: instructions
   emulated (summed over envs); out4[1]: those run on the wave-uniform path;
   out4[2]: instruction passes of the interpreter's waves: one for each
   instruction that a group of lanes ran together on the wave-uniform path,
   and one for each opcode pass of the per-lane path; out4[3]: scheduling
   rounds of those waves (a group formed, then its run on the wave-uniform
   path or a round of per-lane passes).  Active-lane utilisation =
   out4[0] / (64 * out4[2]).  Synchronises. */
int vcs_last_step_counts(vcs_ctx* ctx, uint64_t* out4);

/* Average device time of the named kernel over the timed region: the caller
   brackets steps with vcs_timing(ctx, 1) ... vcs_timing(ctx, 0), then reads
   the mean duration in ms and launch count of kernel `which`
   (0 = interpreter, 1 = render, 2 = render+preprocess, 3 = reset).
   Events are recorded on the stream each kernel is launched on. */
int vcs_timing(vcs_ctx* ctx, int enable);
int vcs_kernel_time(vcs_ctx* ctx, int which, double* mean_ms, uint32_t* launches);

/* ---- batching form: launch shape, autotuner, captured steps ----------------
   The paper runs one GPU thread per emulator and reports two effects of the
   launch on throughput (Section 4, the emulation-only results and "Factors
   affecting the FPS"): low occupancy at small env counts, and divergence of
   envs that share a warp.  The calls below make the shape a parameter, pick
   it by measurement and capture whole steps in a HIP graph.  None of them
   changes any result: outputs and states are identical under every launch
   shape. */
typedef struct {
    uint32_t tile_envs;     /* envs per interpreter wave (one tile): 1, 2, 4, ..., 64.
                               Tiles hold envs of one ROM; fewer envs per wave spread a
                               small batch over more compute units. Default 64. */
    uint32_t workers;       /* 0: one workgroup per tile.  k > 0: a persistent
                               interpreter of k workgroups that take tiles from a device
                               queue until none are left (used only when k is below the
                               tile count).  Default 0. */
    uint32_t render_block;  /* threads per render / observation workgroup: 64, 128, 256
                               or 512.  Default 256. */
} vcs_launch;

/* Set the launch shape (checked as above; VCS_E_INVAL otherwise).  Rebuilds the
   tile table; synchronises.  Graphs captured before are invalidated. */
int vcs_set_launch(vcs_ctx* ctx, const vcs_launch* launch);
int vcs_get_launch(vcs_ctx* ctx, vcs_launch* out);

/* Autotuner.  Times `steps` steps (after one untimed step) of envs 0..n-1
   (n = 0: max_batch) with seeded random actions for each candidate shape,
   one knob at a time: tile_envs (64 and every smaller width that keeps at most
   12 tiles per compute unit), then workers (1, 2, 4, 8 per compute unit, below
   the tile count), then render_block.  Every candidate starts from the same
   env states; afterwards the states, the error bits and the counters are
   restored, so later steps give the results they would have given without
   tuning.  Keeps the fastest shape and returns it with its ms per step; an
   interpreter shape (tile_envs, workers) replaces the current best only when
   at least 3 % faster, so near ties keep the earlier shape (wider tiles, no
   workers: fewer workgroups, which leave compute units to work that overlaps
   the step, such as the previous step's render in captured graphs, and which
   the isolated timing does not see).
   Temporary device buffers (a state snapshot, outputs: frames only if
   want_frames, obs only if want_obs) count against the budget.
   Synchronises. */
int vcs_autotune(vcs_ctx* ctx, uint32_t n, uint32_t steps, int want_frames, int want_obs,
                 vcs_launch* best_out, double* best_ms_out);

/* A HIP graph holding `steps` (1..64) consecutive vcs_step calls with fixed
   arguments: step j reads actions_dev + j*n and writes obs_dev + j*n*84*84,
   reward_dev + j*n, done_dev + j*n and frames_dev + j*n*F*210*160 (obs_dev and
   frames_dev may be NULL).  The caller refills actions_dev between launches.
   A launch enqueues the whole graph on `stream` and gives exactly the results
   of the same vcs_step calls.  VCS_E_STATE after vcs_load_roms, vcs_assign or
   vcs_set_launch on the context.  The graph must be destroyed before its
   context and must not run concurrently with other calls on that context. */
typedef struct vcs_graph vcs_graph;
int vcs_graph_create(vcs_ctx* ctx, const int32_t* env_ids_dev, const uint8_t* actions_dev, uint32_t n,
                     uint32_t steps, uint8_t* obs_dev, int32_t* reward_dev, uint8_t* done_dev,
                     uint8_t* frames_dev, vcs_graph** out);
int vcs_graph_launch(vcs_graph* graph, void* stream);
void vcs_graph_destroy(vcs_graph* graph);

/* ---- frame stack (paper, Section 5, "Memory limitations": agents keep each
   env's last four 84x84 observations; compression is named there as future
   work) ----------------------------------------------------------------
   A stack holds the last `depth` (1..16) observations of every env of the
   context in device memory, as 8-bit gray (bits = 8) or packed to the top
   nibble of each pixel, two pixels per byte (bits = 4: half the memory).
   Created all zero; allocated within the context's budget; destroy it before
   the context. */
typedef struct vcs_stack vcs_stack;
int vcs_stack_create(vcs_ctx* ctx, uint32_t depth, uint32_t bits, vcs_stack** out);
/* Push observations obs_dev[n][84][84] of envs env_ids_dev[0..n) (NULL = envs
   0..n-1; ids must be distinct within a call, as for vcs_step).  An env with
   done_dev[i] != 0 (done_dev may be NULL) starts a new stack: all slots take
   this observation.  out_dev (NULL to skip) receives [n][depth][84][84]
   u8, oldest first, each pixel as stored widened to 8 bits (identity for
   bits = 8, q * 17 for a 4-bit q).  Out-of-range ids are skipped.  Enqueued
   on `stream`; no synchronisation.  Typical use: after vcs_assign / vcs_reset
   push the reset observations with done = 1, then push every step's obs and
   done. */
int vcs_stack_push(vcs_stack* stack, const int32_t* env_ids_dev, uint32_t n, const uint8_t* obs_dev,
                   const uint8_t* done_dev, uint8_t* out_dev, void* stream);
void vcs_stack_destroy(vcs_stack* stack);

/* ---- policy network on the inference path (paper, Section 4: the
   "inference only" load condition, where a policy DNN picks the actions and
   emulation and inference both run on the GPU) ----------------------------
   Fixed architecture (the paper gives none; this is the convolutional trunk
   of the A2C/DQN agents it builds on): input the u8 stack [4][84][84] / 255;
   conv 32 x 8x8 stride 4, conv 64 x 4x4 stride 2, conv 64 x 3x3 stride 1,
   dense 3136 -> 512, each followed by ReLU; dense 512 -> 19 (18 action
   logits, then a value).  bf16 weights and activations, fp32 accumulation on
   the matrix cores, fp32 biases and logits.
   weights_host[l]: bf16 bit patterns, row-major [N_l][K_l]: N = 32, 64, 64,
   512, 19; K = 256, 512, 576, 3136, 512.  Layer 1's reduction index is
   (channel * 8 + ky) * 8 + kx; the others' (ky * KW + kx) * Cin + channel
   (for the dense 3136 -> 512 layer: (y * 7 + x) * 64 + channel of the 7x7x64
   map).  biases_host[l]: float [N_l].  Both are copied; scratch for
   max_batch envs is allocated within the context's budget.  Destroy the
   policy before its context. */
typedef struct vcs_policy vcs_policy;
int vcs_policy_create(vcs_ctx* ctx, const uint16_t* const* weights_host, const float* const* biases_host,
                      vcs_policy** out);
/* Forward pass for stack_dev[n][4][84][84] (n <= max_batch): logits_dev
   (NULL to skip) receives [n][32] floats (entries 0..17 the action logits,
   18 the value, the rest unspecified); actions_dev (NULL to skip) receives,
   per env, the index of the first maximal logit among the 18.  Enqueued on
   `stream`. */
int vcs_policy_act(vcs_policy* policy, const uint8_t* stack_dev, uint32_t n, float* logits_dev, uint8_t* actions_dev,
                   void* stream);
void vcs_policy_destroy(vcs_policy* policy);

const char* vcs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
