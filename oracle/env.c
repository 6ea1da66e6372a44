/*
 * Environment layer of the CPU oracle -- TEST INFRASTRUCTURE (vcs_oracle.h).
 *
 * What the paper fixes (Section 3 and the footnote on raw frames in Section 1):
 *  - frameskip: one env step emulates `frameskip` frames (4 in the paper);
 *  - the observation is the pixelwise maximum of the last two frames of the
 *    step; only those two need rendering;
 *  - episodes restart from a cache of initial states (30 by default), each
 *    made by running 64 start-up frames and up to 30 random no-op frames; at
 *    the end of an episode an env picks one entry at random and copies it.
 *
 * Readings where the paper is silent:
 *  - sticky actions: each frame repeats the previous frame's action when the
 *    counter-based draw R(seed, env, STICKY, step*frameskip + f) >> 32 is
 *    below `sticky_threshold`;
 *  - the step stops early after the frame in which RAM[$D1] != 0 (done);
 *    reward = dec(RAM[$D0] at the stop) - dec(RAM[$D0] at the step start),
 *    dec(b) = 10*(b >> 4) + (b & 15);
 *  - obs = 84x84 exact-area resize of max(gray(F_{k-1}), gray(F_k)) over the
 *    last two frames the step emulated (gray(F_1) when it emulated one);
 *  - frames output: every frame of the step (render mode ALL) or frames
 *    frameskip-2 and frameskip-1 (mode LAST2, the two the paper renders);
 *    frames not emulated because the step stopped early are 0;
 *  - a done env is reset at the end of the same step (eager reset): the
 *    returned obs is that of the cache entry, the returned reward and done
 *    are those of the terminal step;
 *  - a faulted env (undocumented opcode, frame cap, action >= 18) reports
 *    done and is reset the same way; its error bits are kept in a sticky
 *    error word read by oracle_poll_errors;
 *  - cache entry k of ROM r: power-on, run to the first frame end, then
 *    startup_frames NOOP frames, then n_k NOOP frames with
 *    n_k = (R(seed, r, NOOPS, k) >> 32) mod (noop_max + 1); its obs is made
 *    from the last two of those frames;
 *  - reset pick: k = (R(seed, env, RESET, episode_idx) >> 32) mod K, then
 *    episode_idx += 1 and prev_action = NOOP;
 *  - no-ops after the copy (config noop_after_copy, the other reading of the
 *    cache's random no-ops): the entries hold the state startup_frames - 2
 *    frames into the start-up (no no-ops baked in, so all K are alike); a
 *    reset copies one, then runs 2 + n NOOP frames with
 *    n = (R(seed, env, NOOPS_AFTER, episode_idx) >> 32) mod (noop_max + 1)
 *    (no sticky draw, no early stop, the step counter unchanged), and the
 *    observation comes from the last two of them.  Since the start-up frames
 *    are NOOP frames too, the env then holds exactly the state of power-on,
 *    1 + startup_frames + n frames.
 *  RNG: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), used counter-based:
 *  R(seed, id, purpose, n) = mix(mix(mix(mix(seed + G) ^ id) ^ (purpose << 48)) ^ n).
 */
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "machine.h"
#include "vcs_oracle.h"

#define STICKY 1
#define RESET 2
#define NOOPS 3
#define NOOPS_AFTER 4

static const uint64_t GAMMA = 0x9E3779B97F4A7C15ULL;

static uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t oracle_splitmix64_next(uint64_t* state) {
    *state += GAMMA;
    return mix64(*state);
}

uint64_t oracle_rng(uint64_t seed, uint64_t id, uint64_t purpose, uint64_t n) {
    return mix64(mix64(mix64(mix64(seed + GAMMA) ^ id) ^ (purpose << 48)) ^ n);
}

static int n_threads = 0;
int oracle_set_threads(int n) { n_threads = n; return 0; }
int oracle_get_threads(void) {
#ifdef _OPENMP
    return n_threads > 0 ? n_threads : omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------ preprocess */

static int overlap(int a0, int a1, int b0, int b1) {
    int lo = a0 > b0 ? a0 : b0, hi = a1 < b1 ? a1 : b1;
    return hi > lo ? hi - lo : 0;
}

/*
 * obs[i][j] = floor((sum_r sum_c wr(i,r) * wc(j,c) * m[r][c] + 100) / 200)
 * with m = max(gray(f_prev), gray(f_last)), wr(i,r) = |[5i,5i+5) & [2r,2r+2)|
 * (210 rows -> 84, in half rows) and wc(j,c) = |[40j,40j+40) & [21c,21c+21)|
 * (160 columns -> 84, in 1/21 of a pixel): the exact area average, rounded
 * half up.  f_prev may be NULL (one frame).
 */
void oracle_preprocess(const uint8_t* f_prev, const uint8_t* f_last, const uint8_t* lut, uint8_t* obs) {
    for (int i = 0; i < 84; i++) {
        for (int j = 0; j < 84; j++) {
            long sum = 0;
            for (int r = (5 * i) / 2; r <= (5 * i + 4) / 2; r++) {
                int wr = overlap(5 * i, 5 * i + 5, 2 * r, 2 * r + 2);
                for (int c = (40 * j) / 21; c <= (40 * j + 39) / 21; c++) {
                    int wc = overlap(40 * j, 40 * j + 40, 21 * c, 21 * c + 21);
                    int g = lut[f_last[r * 160 + c] >> 1];
                    if (f_prev) {
                        int gp = lut[f_prev[r * 160 + c] >> 1];
                        if (gp > g) g = gp;
                    }
                    sum += (long)wr * wc * g;
                }
            }
            obs[i * 84 + j] = (uint8_t)((sum + 100) / 200);
        }
    }
}

/* ------------------------------------------------------------------- env */

typedef struct {
    uint8_t* data;
    uint32_t size, scheme;
    uint8_t* cache_state;   /* [K][ORC_STATE_BYTES] */
    uint8_t* cache_obs;     /* [K][84*84] */
} ORom;

struct oracle_ctx {
    oracle_config cfg;
    uint32_t n_roms;
    ORom* roms;
    OMachine* envs;
    int assigned;
    uint32_t err_bits;
    uint32_t err_first;
};

int oracle_create(const oracle_config* cfg, oracle_ctx** out) {
    if (!cfg || !out || cfg->num_envs == 0 || cfg->frameskip == 0 || cfg->reset_cache_k == 0 ||
        cfg->render_mode > 1 || (cfg->noop_after_copy && cfg->startup_frames < 2))
        return ORC_E_INVAL;
    oracle_ctx* c = (oracle_ctx*)calloc(1, sizeof(*c));
    if (!c) return ORC_E_NOMEM;
    c->cfg = *cfg;
    c->envs = (OMachine*)calloc(cfg->num_envs, sizeof(OMachine));
    if (!c->envs) { free(c); return ORC_E_NOMEM; }
    c->err_first = 0xFFFFFFFFu;
    *out = c;
    return ORC_OK;
}

static void free_roms(oracle_ctx* c) {
    for (uint32_t r = 0; r < c->n_roms; r++) {
        free(c->roms[r].data);
        free(c->roms[r].cache_state);
        free(c->roms[r].cache_obs);
    }
    free(c->roms);
    c->roms = NULL;
    c->n_roms = 0;
}

void oracle_destroy(oracle_ctx* c) {
    if (!c) return;
    free_roms(c);
    free(c->envs);
    free(c);
}

int oracle_load_roms(oracle_ctx* c, uint32_t n_roms, const uint8_t* const* roms, const uint32_t* bytes,
                     const uint32_t* schemes) {
    if (!c || !roms || !bytes || !schemes || n_roms == 0 || n_roms > 65535) return ORC_E_INVAL;
    for (uint32_t r = 0; r < n_roms; r++) {
        if (!roms[r]) return ORC_E_INVAL;
        if (!m_rom_size_ok(bytes[r], schemes[r])) return ORC_E_ROM;
    }
    free_roms(c);
    c->roms = (ORom*)calloc(n_roms, sizeof(ORom));
    if (!c->roms) return ORC_E_NOMEM;
    c->n_roms = n_roms;
    for (uint32_t r = 0; r < n_roms; r++) {
        c->roms[r].data = (uint8_t*)malloc(bytes[r]);
        if (!c->roms[r].data) return ORC_E_NOMEM;
        memcpy(c->roms[r].data, roms[r], bytes[r]);
        c->roms[r].size = bytes[r];
        c->roms[r].scheme = schemes[r];
    }
    c->assigned = 0;
    return ORC_OK;
}

/* Build cache entry k of ROM r (power-on, start-up and no-op frames). */
static void build_cache_entry(oracle_ctx* c, uint32_t r, uint32_t k) {
    ORom* rom = &c->roms[r];
    OMachine m;
    m_power_on(&m, rom->data, rom->size, rom->scheme);
    m.track_cx = c->cfg.collisions ? 1 : 0;
    m_set_action(&m, 0);
    uint32_t noops = (uint32_t)((oracle_rng(c->cfg.seed, r, NOOPS, k) >> 32) % (c->cfg.noop_max + 1));
    uint32_t total = 1 + c->cfg.startup_frames + noops;   /* frame 0 + start-up + no-ops */
    if (c->cfg.noop_after_copy) total = 1 + c->cfg.startup_frames - 2;   /* the reset runs the rest */
    uint8_t* fb[2];
    fb[0] = (uint8_t*)malloc(2 * 210 * 160);
    fb[1] = fb[0] + 210 * 160;
    uint32_t last_rendered = 0;
    for (uint32_t f = 0; f < total; f++) {
        uint8_t* target = (f + 2 >= total) ? fb[f & 1] : NULL;
        m_run_frame(&m, target, NULL);
        if (target) last_rendered++;
    }
    m.rom_id = r;
    m.prev_action = 0;
    m.err = 0;
    m.step_idx = 0;
    m.episode_idx = 0;
    uint8_t* obs = rom->cache_obs + (size_t)k * 84 * 84;
    if (total >= 2)
        oracle_preprocess(fb[(total - 2) & 1], fb[(total - 1) & 1], c->cfg.gray_lut, obs);
    else
        oracle_preprocess(NULL, fb[(total - 1) & 1], c->cfg.gray_lut, obs);
    m_to_record(&m, rom->cache_state + (size_t)k * ORC_STATE_BYTES);
    (void)last_rendered;
    free(fb[0]);
}

/* Copy a cache entry into env e (eager reset) and return the cache obs; with
   no-ops after the copy, run them and return the obs of their last two
   frames.  Returns the error bits of those frames. */
static uint32_t reset_env(oracle_ctx* c, uint32_t e, uint8_t* obs_out) {
    OMachine* m = &c->envs[e];
    uint32_t r = m->rom_id;
    uint32_t K = c->cfg.reset_cache_k;
    uint32_t k = (uint32_t)((oracle_rng(c->cfg.seed, e, RESET, m->episode_idx) >> 32) % K);
    uint32_t step = m->step_idx, episode = m->episode_idx;
    ORom* rom = &c->roms[r];
    m_from_record(m, rom->cache_state + (size_t)k * ORC_STATE_BYTES);
    m->rom = rom->data;
    m->rom_size = rom->size;
    m->scheme = rom->scheme;
    m->fb = NULL;
    m->rom_id = r;
    m->step_idx = step;
    m->episode_idx = episode + 1;
    m->prev_action = 0;
    m->err = 0;
    m_set_action(m, 0);
    if (!c->cfg.noop_after_copy) {
        if (obs_out) memcpy(obs_out, rom->cache_obs + (size_t)k * 84 * 84, 84 * 84);
        return 0;
    }
    uint32_t n = (uint32_t)((oracle_rng(c->cfg.seed, e, NOOPS_AFTER, episode) >> 32) % (c->cfg.noop_max + 1));
    uint32_t total = 2 + n;
    int have[2] = {0, 0};                 /* slot s: frame total - 2 + s, emulated */
    uint8_t* fb = (uint8_t*)calloc(2, 210 * 160);
    for (uint32_t f = 0; f < total; f++) {
        int slot = (int)f - (int)(total - 2);
        m_run_frame(m, slot >= 0 ? fb + (size_t)slot * 210 * 160 : NULL, NULL);
        if (slot >= 0) have[slot] = 1;
        if (m->err) break;
    }
    if (obs_out) {
        if (have[0] && have[1]) oracle_preprocess(fb, fb + 210 * 160, c->cfg.gray_lut, obs_out);
        else if (have[0] || have[1]) oracle_preprocess(NULL, fb + (have[1] ? 210 * 160 : 0), c->cfg.gray_lut, obs_out);
        else memset(obs_out, 0, 84 * 84);
    }
    free(fb);
    return m->err;
}

int oracle_assign(oracle_ctx* c, const uint16_t* env_rom) {
    if (!c || !env_rom || c->n_roms == 0) return ORC_E_INVAL;
    for (uint32_t e = 0; e < c->cfg.num_envs; e++)
        if (env_rom[e] >= c->n_roms) return ORC_E_INVAL;
    uint32_t K = c->cfg.reset_cache_k;
    for (uint32_t r = 0; r < c->n_roms; r++) {
        free(c->roms[r].cache_state);
        free(c->roms[r].cache_obs);
        c->roms[r].cache_state = (uint8_t*)calloc(K, ORC_STATE_BYTES);
        c->roms[r].cache_obs = (uint8_t*)calloc(K, 84 * 84);
        if (!c->roms[r].cache_state || !c->roms[r].cache_obs) return ORC_E_NOMEM;
    }
    long total = (long)c->n_roms * K;
#pragma omp parallel for schedule(dynamic) num_threads(oracle_get_threads())
    for (long i = 0; i < total; i++) build_cache_entry(c, (uint32_t)(i / K), (uint32_t)(i % K));
    for (uint32_t e = 0; e < c->cfg.num_envs; e++) {
        memset(&c->envs[e], 0, sizeof(OMachine));
        c->envs[e].rom_id = env_rom[e];
        reset_env(c, e, NULL);
    }
    c->assigned = 1;
    c->err_bits = 0;
    c->err_first = 0xFFFFFFFFu;
    return ORC_OK;
}

static int check_ids(const oracle_ctx* c, const int32_t* ids, uint32_t n) {
    if (n > c->cfg.num_envs) return ORC_E_INVAL;
    if (!ids) return ORC_OK;
    uint8_t* seen = (uint8_t*)calloc(c->cfg.num_envs, 1);
    if (!seen) return ORC_E_NOMEM;
    int rc = ORC_OK;
    for (uint32_t i = 0; i < n; i++) {
        if (ids[i] < 0 || (uint32_t)ids[i] >= c->cfg.num_envs || seen[ids[i]]) { rc = ORC_E_INVAL; break; }
        seen[ids[i]] = 1;
    }
    free(seen);
    return rc;
}

int oracle_reset(oracle_ctx* c, const int32_t* ids, uint32_t n, uint8_t* obs) {
    if (!c || !c->assigned) return ORC_E_STATE;
    int rc = check_ids(c, ids, n);
    if (rc) return rc;
    for (uint32_t i = 0; i < n; i++) {
        uint32_t e = ids ? (uint32_t)ids[i] : i;
        reset_env(c, e, obs ? obs + (size_t)i * 84 * 84 : NULL);
    }
    return ORC_OK;
}

static int bcd_value(uint8_t b) { return 10 * (b >> 4) + (b & 15); }

/* One env step of env e: returns its error bits. */
static uint32_t step_env(oracle_ctx* c, uint32_t e, uint8_t action, uint8_t* obs, int32_t* reward,
                         uint8_t* done, uint8_t* frames, int render) {
    OMachine* m = &c->envs[e];
    uint32_t fs = c->cfg.frameskip;
    uint32_t n_slots = c->cfg.render_mode == ORC_RENDER_LAST2 ? 2 : fs;
    size_t fsz = 210 * 160;
    uint8_t* fb = (uint8_t*)calloc((size_t)fs, fsz);
    uint32_t errs = 0;
    int is_done = 0;
    uint32_t k = 0;
    uint8_t score0 = m->ram[0x50];
    if (action >= 18) {
        m->err |= ORC_ERR_BAD_ACTION;
        is_done = 1;
    } else {
        uint8_t prev = m->prev_action;
        for (uint32_t f = 0; f < fs; f++) {
            uint8_t eff = action;
            if (c->cfg.sticky_threshold) {
                uint64_t draw = oracle_rng(c->cfg.seed, e, STICKY, (uint64_t)m->step_idx * fs + f) >> 32;
                if (draw < c->cfg.sticky_threshold) eff = prev;
            }
            m_set_action(m, eff);
            m_run_frame(m, (render || frames) ? fb + (size_t)f * fsz : NULL, NULL);
            prev = eff;
            k++;
            if (m->err || m->ram[0x51] != 0) { is_done = 1; break; }
        }
        m->prev_action = prev;
    }
    *reward = bcd_value(m->ram[0x50]) - bcd_value(score0);
    *done = (uint8_t)is_done;
    errs = m->err;
    if (frames) {
        uint8_t* out = frames;
        memset(out, 0, (size_t)n_slots * fsz);
        if (c->cfg.render_mode == ORC_RENDER_ALL) {
            memcpy(out, fb, (size_t)k * fsz);
        } else {
            /* the two frames selective rendering keeps: fs-2 and fs-1 (0 if not emulated) */
            for (int s = 0; s < 2; s++) {
                int f = (int)fs - 2 + s;
                if (f >= 0 && (uint32_t)f < k) memcpy(out + (size_t)s * fsz, fb + (size_t)f * fsz, fsz);
            }
        }
    }
    if (render && obs && k >= 1)
        oracle_preprocess(k >= 2 ? fb + (size_t)(k - 2) * fsz : NULL, fb + (size_t)(k - 1) * fsz,
                          c->cfg.gray_lut, obs);
    else if (obs && k == 0)
        memset(obs, 0, 84 * 84);
    m->step_idx++;
    if (is_done) errs |= reset_env(c, e, obs);
    free(fb);
    return errs;
}

int oracle_step(oracle_ctx* c, const int32_t* ids, const uint8_t* actions, uint32_t n, uint8_t* obs,
                int32_t* reward, uint8_t* done, uint8_t* frames, int render) {
    if (!c || !c->assigned) return ORC_E_STATE;
    if (!actions || !reward || !done) return ORC_E_INVAL;
    int rc = check_ids(c, ids, n);
    if (rc) return rc;
    uint32_t n_slots = c->cfg.render_mode == ORC_RENDER_LAST2 ? 2 : c->cfg.frameskip;
    uint32_t* errs = (uint32_t*)calloc(n ? n : 1, sizeof(uint32_t));
#pragma omp parallel for schedule(dynamic, 1) num_threads(oracle_get_threads())
    for (long i = 0; i < (long)n; i++) {
        uint32_t e = ids ? (uint32_t)ids[i] : (uint32_t)i;
        errs[i] = step_env(c, e, actions[i], obs ? obs + (size_t)i * 84 * 84 : NULL, reward + i, done + i,
                           frames ? frames + (size_t)i * n_slots * 210 * 160 : NULL, render);
    }
    for (uint32_t i = 0; i < n; i++) {
        if (!errs[i]) continue;
        uint32_t e = ids ? (uint32_t)ids[i] : i;
        c->err_bits |= errs[i];
        if (e < c->err_first) c->err_first = e;
    }
    free(errs);
    return ORC_OK;
}

int oracle_get_state(oracle_ctx* c, uint32_t env, uint8_t* out) {
    if (!c || !out || env >= c->cfg.num_envs) return ORC_E_INVAL;
    m_to_record(&c->envs[env], out);
    return ORC_OK;
}

int oracle_set_state(oracle_ctx* c, uint32_t env, const uint8_t* in) {
    if (!c || !in || env >= c->cfg.num_envs || !c->assigned) return ORC_E_INVAL;
    uint32_t r = in[180] | (in[181] << 8) | (in[182] << 16) | ((uint32_t)in[183] << 24);
    if (r >= c->n_roms) return ORC_E_INVAL;
    OMachine* m = &c->envs[env];
    m_from_record(m, in);
    m->track_cx = c->cfg.collisions ? 1 : 0;
    m->rom = c->roms[r].data;
    m->rom_size = c->roms[r].size;
    m->scheme = c->roms[r].scheme;
    m->fb = NULL;
    return ORC_OK;
}

int oracle_get_cache(oracle_ctx* c, uint32_t rom, uint32_t k, uint8_t* state, uint8_t* obs) {
    if (!c || !c->assigned || rom >= c->n_roms || k >= c->cfg.reset_cache_k) return ORC_E_INVAL;
    if (state) memcpy(state, c->roms[rom].cache_state + (size_t)k * ORC_STATE_BYTES, ORC_STATE_BYTES);
    if (obs) memcpy(obs, c->roms[rom].cache_obs + (size_t)k * 84 * 84, 84 * 84);
    return ORC_OK;
}

int oracle_poll_errors(oracle_ctx* c, uint32_t* first_env, uint32_t* bits) {
    if (!c || !first_env || !bits) return ORC_E_INVAL;
    *first_env = c->err_first;
    *bits = c->err_bits;
    c->err_bits = 0;
    c->err_first = 0xFFFFFFFFu;
    return ORC_OK;
}

/* ------------------------------------------------------ bare machine */

int oracle_power_on(const uint8_t* rom, uint32_t bytes, uint32_t scheme, uint8_t* state) {
    if (!rom || !state) return ORC_E_INVAL;
    if (!m_rom_size_ok(bytes, scheme)) return ORC_E_ROM;
    OMachine m;
    m_power_on(&m, rom, bytes, scheme);
    m_to_record(&m, state);
    return ORC_OK;
}

static void load_bare(OMachine* m, const uint8_t* state, const uint8_t* rom, uint32_t bytes, uint32_t scheme) {
    memset(m, 0, sizeof(*m));
    m_from_record(m, state);
    m->rom = rom;
    m->rom_size = bytes;
    m->scheme = scheme;
}

/* Run n instructions (frame ends do not stop it; a fault does). */
int oracle_run_instructions(uint8_t* state, const uint8_t* rom, uint32_t bytes, uint32_t scheme,
                            uint32_t n_instr, uint32_t action) {
    if (!state || !rom) return ORC_E_INVAL;
    OMachine m;
    load_bare(&m, state, rom, bytes, scheme);
    m_set_action(&m, action);
    uint32_t done = 0;
    for (; done < n_instr; done++) {
        int why = m_step_instruction(&m);
        if (why == END_CAP || why == END_ILLEGAL) break;
    }
    m_to_record(&m, state);
    return (int)done;
}

int oracle_batch_instructions(uint8_t* states, uint32_t n_states, const uint8_t* rom, uint32_t bytes,
                              uint32_t scheme, uint32_t n_instr) {
    if (!states || !rom) return ORC_E_INVAL;
#pragma omp parallel for schedule(static) num_threads(oracle_get_threads())
    for (long i = 0; i < (long)n_states; i++)
        oracle_run_instructions(states + (size_t)i * ORC_STATE_BYTES, rom, bytes, scheme, n_instr, 0);
    return ORC_OK;
}

int oracle_run_frames(uint8_t* state, const uint8_t* rom, uint32_t bytes, uint32_t scheme, uint32_t n_frames,
                      const uint8_t* actions, uint8_t* frames, uint64_t* frame_end_cycle) {
    if (!state || !rom) return ORC_E_INVAL;
    OMachine m;
    load_bare(&m, state, rom, bytes, scheme);
    uint32_t f = 0;
    for (; f < n_frames; f++) {
        m_set_action(&m, actions ? actions[f] : 0);
        int why = m_run_frame(&m, frames ? frames + (size_t)f * 210 * 160 : NULL,
                              frame_end_cycle ? frame_end_cycle + f : NULL);
        if (why != END_VSYNC) { f++; break; }
    }
    m_to_record(&m, state);
    return (int)f;
}
