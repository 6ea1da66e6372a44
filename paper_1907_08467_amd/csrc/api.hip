// vcs355 C ABI: context, device memory plan and the step/reset pipelines.
//
// Per step (all on the caller's stream, no host synchronisation):
//   [ids given]  validate ids, count per ROM, lay out ROM-homogeneous tiles
//   k_interp           frameskip frames per env, row logs for rendered frames
//   k_render_frames    frames that only go to the frames output (mode ALL)
//   k_render_obs       the last two frames -> frames output and 84x84 obs
//   k_reset            envs that ended restart from the reset cache
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/vcs355.h"
#include "vcs_device.h"

using namespace vcs;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIP_OK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(VCS_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct TimedLaunch {
    int kind;
    hipEvent_t start, stop;
};

}  // namespace

struct vcs_ctx {
    vcs_config cfg{};
    uint32_t max_batch = 0;
    uint32_t n_slots = 0;
    size_t allocated = 0;
    std::vector<void*> owned;

    // ROMs
    uint32_t n_roms = 0;
    uint8_t* d_roms = nullptr;
    uint32_t* d_schemes = nullptr;
    std::vector<uint32_t> h_schemes;
    std::vector<uint8_t> h_roms;   // [n_roms][kRomSlot]

    // envs
    DevEnv* d_envs = nullptr;
    uint16_t* d_env_rom = nullptr;
    std::vector<uint16_t> h_env_rom;
    bool assigned = false;

    // reset cache
    DevEnv* d_cache_state = nullptr;
    uint8_t* d_cache_obs = nullptr;

    // tiles
    Tile* d_tiles_all = nullptr;
    uint32_t n_tiles_all = 0;
    uint32_t* d_n_tiles_all = nullptr;
    Tile* d_tiles = nullptr;
    uint32_t tiles_cap = 0;
    uint32_t* d_n_tiles = nullptr;
    uint32_t* d_counts = nullptr;   // [n_roms] x 3: counts, offsets, fill
    uint32_t* d_claim = nullptr;
    uint8_t* d_valid = nullptr;
    uint32_t tag = 0;

    // per-step scratch
    uint8_t* d_logs = nullptr;
    StepInfo* d_info = nullptr;
    uint32_t* d_err = nullptr;
    unsigned long long* d_instr = nullptr;
    uint8_t* d_gray = nullptr;

    // timing
    bool timing = false;
    std::vector<TimedLaunch> timed;
};

namespace {

int dev_alloc(vcs_ctx* c, void** p, size_t bytes, const char* what) {
    if (c->cfg.hbm_budget_bytes && c->allocated + bytes > c->cfg.hbm_budget_bytes)
        return fail(VCS_E_BUDGET, std::string("HBM budget exceeded allocating ") + what);
    if (hipMalloc(p, bytes ? bytes : 16) != hipSuccess) return fail(VCS_E_NOMEM, std::string("hipMalloc failed: ") + what);
    c->allocated += bytes;
    c->owned.push_back(*p);
    return VCS_OK;
}

void dev_free(vcs_ctx* c, void* p, size_t bytes) {
    if (!p) return;
    (void)hipFree(p);
    c->allocated -= std::min(c->allocated, bytes);
    c->owned.erase(std::remove(c->owned.begin(), c->owned.end(), p), c->owned.end());
}

template <typename T>
int alloc_n(vcs_ctx* c, T** p, size_t n, const char* what) {
    return dev_alloc(c, reinterpret_cast<void**>(p), n * sizeof(T), what);
}

void begin_timed(vcs_ctx* c, int kind, hipStream_t s) {
    if (!c->timing) return;
    TimedLaunch t{kind, nullptr, nullptr};
    (void)hipEventCreate(&t.start);
    (void)hipEventCreate(&t.stop);
    (void)hipEventRecord(t.start, s);
    c->timed.push_back(t);
}
void end_timed(vcs_ctx* c, hipStream_t s) {
    if (!c->timing) return;
    (void)hipEventRecord(c->timed.back().stop, s);
}
void clear_timed(vcs_ctx* c) {
    for (auto& t : c->timed) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    c->timed.clear();
}

// power-on state of a console with ROM `r`
DevEnv power_on(const vcs_ctx* c, uint32_t r) {
    DevEnv e;
    std::memset(&e, 0, sizeof(e));
    const uint8_t* rom = c->h_roms.data() + (size_t)r * kRomSlot;
    const uint32_t bank = c->h_schemes[r] == VCS_BANK_F8 ? 1 : 0;
    e.sp = 0xFD;
    e.p = 0x24;
    e.bank = (uint8_t)bank;
    e.pc = (uint16_t)(rom[(bank << 12) | 0xFFC] | (rom[(bank << 12) | 0xFFD] << 8));
    e.tv = 0;
    e.tshift = 10;
    e.tbase = 0;
    e.rom_id = r;
    return e;
}

// GPU record -> exchange record (vcs355.h)
void to_record(const DevEnv& e, uint8_t* out) {
    std::memset(out, 0, VCS_STATE_BYTES);
    out[0] = e.a; out[1] = e.x; out[2] = e.y; out[3] = e.sp; out[4] = e.p; out[5] = e.bank;
    std::memcpy(out + 6, &e.pc, 2);
    std::memcpy(out + 8, &e.cycle, 8);
    std::memcpy(out + 16, &e.frame_line0, 8);
    int64_t ev = (int64_t)e.cycle - e.tbase;
    if (ev < 0) ev = 0;
    const int64_t lim = (int64_t)(e.tv + 1) << e.tshift;
    const bool expired = ev >= lim;
    out[24] = expired ? (uint8_t)((0xFF - (ev - lim)) & 0xFF) : (uint8_t)(e.tv - (ev >> e.tshift));
    out[25] = expired ? 1 : 0;
    const uint16_t interval = (uint16_t)(1u << e.tshift);
    std::memcpy(out + 26, &interval, 2);
    const uint16_t phase = expired ? 0 : (uint16_t)(ev & (interval - 1));
    std::memcpy(out + 28, &phase, 2);
    std::memcpy(out + 32, e.ram, 128);
    const uint8_t regs[18] = {e.vsync, e.tia[R_VBLANK], e.tia[R_COLUP0], e.tia[R_COLUP1], e.tia[R_COLUPF],
                              e.tia[R_COLUBK], e.tia[R_CTRLPF], e.tia[R_REFP0], e.tia[R_REFP1], e.tia[R_PF0],
                              e.tia[R_PF1], e.tia[R_PF2], e.tia[R_GRP0], e.tia[R_GRP1], e.hmp0, e.hmp1,
                              e.tia[R_P0X], e.tia[R_P1X]};
    std::memcpy(out + 160, regs, 18);
    std::memcpy(out + 180, &e.rom_id, 4);
    std::memcpy(out + 184, &e.step_idx, 4);
    std::memcpy(out + 188, &e.episode_idx, 4);
    out[192] = e.prev_action;
    out[194] = e.err;
    std::memcpy(out + 200, &e.instr, 8);
}

int from_record(const uint8_t* in, DevEnv* e) {
    std::memset(e, 0, sizeof(*e));
    e->a = in[0]; e->x = in[1]; e->y = in[2]; e->sp = in[3]; e->p = in[4]; e->bank = in[5];
    std::memcpy(&e->pc, in + 6, 2);
    std::memcpy(&e->cycle, in + 8, 8);
    std::memcpy(&e->frame_line0, in + 16, 8);
    uint16_t interval, phase;
    std::memcpy(&interval, in + 26, 2);
    std::memcpy(&phase, in + 28, 2);
    int sh = -1;
    if (interval == 1) sh = 0;
    if (interval == 8) sh = 3;
    if (interval == 64) sh = 6;
    if (interval == 1024) sh = 10;
    if (sh < 0 || phase >= interval) return -1;
    e->tshift = (uint8_t)sh;
    if (!in[25]) {
        e->tv = in[24];
        e->tbase = (int64_t)e->cycle - phase;
    } else {
        e->tv = 0;
        e->tbase = (int64_t)e->cycle - (int64_t)interval - (int64_t)((0xFF - in[24]) & 0xFF);
    }
    std::memcpy(e->ram, in + 32, 128);
    const uint8_t* r = in + 160;
    e->vsync = r[0]; e->tia[R_VBLANK] = r[1]; e->tia[R_COLUP0] = r[2]; e->tia[R_COLUP1] = r[3];
    e->tia[R_COLUPF] = r[4]; e->tia[R_COLUBK] = r[5]; e->tia[R_CTRLPF] = r[6]; e->tia[R_REFP0] = r[7];
    e->tia[R_REFP1] = r[8]; e->tia[R_PF0] = r[9]; e->tia[R_PF1] = r[10]; e->tia[R_PF2] = r[11];
    e->tia[R_GRP0] = r[12]; e->tia[R_GRP1] = r[13]; e->hmp0 = r[14]; e->hmp1 = r[15];
    e->tia[R_P0X] = r[16]; e->tia[R_P1X] = r[17];
    std::memcpy(&e->rom_id, in + 180, 4);
    std::memcpy(&e->step_idx, in + 184, 4);
    std::memcpy(&e->episode_idx, in + 188, 4);
    e->prev_action = in[192];
    e->err = in[194];
    std::memcpy(&e->instr, in + 200, 8);
    return 0;
}

// Build ROM-homogeneous tiles on the device for the ids of one call.
int build_tiles(vcs_ctx* c, const int32_t* ids, uint32_t n, int32_t* reward, uint8_t* done, hipStream_t s,
                uint32_t* grid) {
    uint32_t* counts = c->d_counts;
    uint32_t* offsets = c->d_counts + c->n_roms;
    uint32_t* fill = c->d_counts + 2 * c->n_roms;
    launch_fill_u32(counts, c->n_roms, 0, s);
    launch_validate(ids, n, c->cfg.num_envs, c->d_env_rom, c->d_claim, c->tag++, counts, c->d_valid, c->d_info,
                    reward, done, c->d_err, s);
    launch_tile_layout(counts, c->n_roms, offsets, fill, c->d_tiles, c->d_n_tiles, s);
    launch_tile_fill(ids, n, c->d_env_rom, c->d_valid, offsets, fill, c->d_tiles, s);
    *grid = (n + kLanes - 1) / kLanes + c->n_roms;
    HIP_OK(hipGetLastError());
    return VCS_OK;
}

}  // namespace

extern "C" {

const char* vcs_last_error(void) { return g_err.c_str(); }

int vcs_create(const vcs_config* cfg, vcs_ctx** out) {
    if (!cfg || !out) return fail(VCS_E_INVAL, "null argument");
    *out = nullptr;
    if (cfg->num_envs == 0) return fail(VCS_E_INVAL, "num_envs must be >= 1");
    if (cfg->frameskip == 0 || cfg->frameskip > 255) return fail(VCS_E_INVAL, "frameskip must be in [1, 255]");
    if (cfg->render_mode > VCS_RENDER_LAST2) return fail(VCS_E_INVAL, "bad render_mode");
    if (cfg->render_mode == VCS_RENDER_ALL && cfg->frameskip > 8)
        return fail(VCS_E_INVAL, "render_mode ALL supports frameskip <= 8");
    if (cfg->reset_cache_k == 0) return fail(VCS_E_INVAL, "reset_cache_k must be >= 1");
    if (cfg->max_batch > cfg->num_envs) return fail(VCS_E_INVAL, "max_batch > num_envs");
    if (1 + cfg->startup_frames + cfg->noop_max > 65535) return fail(VCS_E_INVAL, "cache build too long");
    int ndev = 0;
    HIP_OK(hipGetDeviceCount(&ndev));
    if (cfg->device < 0 || cfg->device >= ndev) return fail(VCS_E_INVAL, "bad device ordinal");
    HIP_OK(hipSetDevice(cfg->device));

    vcs_ctx* c = new vcs_ctx();
    c->cfg = *cfg;
    c->max_batch = cfg->max_batch ? cfg->max_batch : cfg->num_envs;
    c->n_slots = cfg->render_mode == VCS_RENDER_ALL ? cfg->frameskip : 2;
    int rc = VCS_OK;
    const size_t B = c->max_batch;
    if (!rc) rc = alloc_n(c, &c->d_envs, cfg->num_envs, "env state");
    if (!rc) rc = alloc_n(c, &c->d_env_rom, cfg->num_envs, "env rom");
    if (!rc) rc = alloc_n(c, &c->d_claim, cfg->num_envs, "id claims");
    if (!rc) rc = alloc_n(c, &c->d_logs, B * c->n_slots * kFrameLogBytes, "row logs");
    if (!rc) rc = alloc_n(c, &c->d_info, B, "step info");
    if (!rc) rc = alloc_n(c, &c->d_valid, B, "id validity");
    if (!rc) rc = alloc_n(c, &c->d_err, 2, "error word");
    if (!rc) rc = alloc_n(c, &c->d_instr, 2, "instruction counters");
    if (!rc) rc = alloc_n(c, &c->d_gray, 128, "gray table");
    if (!rc) rc = alloc_n(c, &c->d_n_tiles, 1, "tile count");
    if (!rc) rc = alloc_n(c, &c->d_n_tiles_all, 1, "tile count");
    if (rc) {
        vcs_destroy(c);
        return rc;
    }
    if (hipMemcpy(c->d_gray, cfg->gray_lut, 128, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(c->d_claim, 0xFF, (size_t)cfg->num_envs * 4) != hipSuccess ||
        hipMemset(c->d_err, 0, 4) != hipSuccess || hipMemset(c->d_err + 1, 0xFF, 4) != hipSuccess ||
        hipMemset(c->d_envs, 0, (size_t)cfg->num_envs * sizeof(DevEnv)) != hipSuccess) {
        vcs_destroy(c);
        return fail(VCS_E_HIP, "initial device copies failed");
    }
    *out = c;
    return VCS_OK;
}

void vcs_destroy(vcs_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->cfg.device);
    (void)hipDeviceSynchronize();
    clear_timed(c);
    for (void* p : c->owned) (void)hipFree(p);
    delete c;
}

int vcs_load_roms(vcs_ctx* c, uint32_t n_roms, const uint8_t* const* rom_host, const uint32_t* rom_bytes,
                  const uint32_t* scheme) {
    if (!c || !rom_host || !rom_bytes || !scheme) return fail(VCS_E_INVAL, "null argument");
    if (n_roms == 0 || n_roms > 65535) return fail(VCS_E_INVAL, "n_roms must be in [1, 65535]");
    for (uint32_t r = 0; r < n_roms; ++r) {
        if (!rom_host[r]) return fail(VCS_E_INVAL, "null ROM pointer");
        const bool ok4 = scheme[r] == VCS_BANK_4K && rom_bytes[r] == 4096;
        const bool ok8 = scheme[r] == VCS_BANK_F8 && rom_bytes[r] == 8192;
        if (!ok4 && !ok8) return fail(VCS_E_ROM, "ROM " + std::to_string(r) + ": need 4096 B (4K) or 8192 B (F8)");
    }
    HIP_OK(hipSetDevice(c->cfg.device));
    HIP_OK(hipDeviceSynchronize());
    dev_free(c, c->d_roms, (size_t)c->n_roms * kRomSlot);
    dev_free(c, c->d_schemes, (size_t)c->n_roms * 4);
    dev_free(c, c->d_counts, (size_t)c->n_roms * 12);
    dev_free(c, c->d_tiles, (size_t)c->tiles_cap * sizeof(Tile));
    c->d_roms = nullptr; c->d_schemes = nullptr; c->d_counts = nullptr; c->d_tiles = nullptr;
    c->assigned = false;
    c->n_roms = n_roms;
    c->h_roms.assign((size_t)n_roms * kRomSlot, 0);
    c->h_schemes.assign(scheme, scheme + n_roms);
    for (uint32_t r = 0; r < n_roms; ++r) std::memcpy(c->h_roms.data() + (size_t)r * kRomSlot, rom_host[r], rom_bytes[r]);
    int rc = alloc_n(c, &c->d_roms, (size_t)n_roms * kRomSlot, "ROMs");
    if (!rc) rc = alloc_n(c, &c->d_schemes, n_roms, "ROM schemes");
    if (!rc) rc = alloc_n(c, &c->d_counts, (size_t)n_roms * 3, "tile counters");
    c->tiles_cap = (c->max_batch + kLanes - 1) / kLanes + n_roms;
    if (!rc) rc = alloc_n(c, &c->d_tiles, c->tiles_cap, "tiles");
    if (rc) return rc;
    HIP_OK(hipMemcpy(c->d_roms, c->h_roms.data(), c->h_roms.size(), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(c->d_schemes, c->h_schemes.data(), n_roms * 4, hipMemcpyHostToDevice));
    return VCS_OK;
}

int vcs_assign(vcs_ctx* c, const uint16_t* env_rom_host) {
    if (!c || !env_rom_host) return fail(VCS_E_INVAL, "null argument");
    if (c->n_roms == 0) return fail(VCS_E_STATE, "vcs_load_roms first");
    const uint32_t N = c->cfg.num_envs, R = c->n_roms, K = c->cfg.reset_cache_k;
    for (uint32_t e = 0; e < N; ++e)
        if (env_rom_host[e] >= R) return fail(VCS_E_INVAL, "env " + std::to_string(e) + " has no such ROM");
    HIP_OK(hipSetDevice(c->cfg.device));
    c->h_env_rom.assign(env_rom_host, env_rom_host + N);
    HIP_OK(hipMemcpy(c->d_env_rom, env_rom_host, (size_t)N * 2, hipMemcpyHostToDevice));

    // tiles over all envs, ROM by ROM
    std::vector<Tile> tiles;
    {
        std::vector<std::vector<int32_t>> by_rom(R);
        for (uint32_t e = 0; e < N; ++e) by_rom[env_rom_host[e]].push_back((int32_t)e);
        for (uint32_t r = 0; r < R; ++r) {
            for (size_t i = 0; i < by_rom[r].size(); i += kLanes) {
                Tile t;
                std::memset(&t, 0xFF, sizeof(t));
                t.rom = (int32_t)r;
                t.count = (int32_t)std::min<size_t>(kLanes, by_rom[r].size() - i);
                for (int l = 0; l < t.count; ++l) {
                    t.env[l] = by_rom[r][i + l];
                    t.out[l] = by_rom[r][i + l];
                }
                tiles.push_back(t);
            }
        }
    }
    dev_free(c, c->d_tiles_all, (size_t)c->n_tiles_all * sizeof(Tile));
    c->d_tiles_all = nullptr;
    c->n_tiles_all = (uint32_t)tiles.size();
    int rc = alloc_n(c, &c->d_tiles_all, tiles.size(), "tiles (all envs)");
    if (rc) return rc;
    HIP_OK(hipMemcpy(c->d_tiles_all, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(c->d_n_tiles_all, &c->n_tiles_all, 4, hipMemcpyHostToDevice));

    // ---- reset cache: K entries per ROM
    const uint32_t M = R * K;
    dev_free(c, c->d_cache_state, (size_t)M * sizeof(DevEnv));
    dev_free(c, c->d_cache_obs, (size_t)M * kObsBytes);
    c->d_cache_state = nullptr;
    c->d_cache_obs = nullptr;
    rc = alloc_n(c, &c->d_cache_state, M, "reset cache states");
    if (!rc) rc = alloc_n(c, &c->d_cache_obs, (size_t)M * kObsBytes, "reset cache obs");
    if (rc) return rc;
    std::vector<DevEnv> cst(M);
    std::vector<uint16_t> nfr(M);
    std::vector<Tile> ctiles;
    for (uint32_t r = 0; r < R; ++r) {
        const DevEnv p0 = power_on(c, r);
        for (uint32_t k = 0; k < K; ++k) {
            cst[r * K + k] = p0;
            const uint64_t draw = rng_draw(rng_prefix(c->cfg.seed, r, kNoopPurpose), k);
            const uint32_t noops = (uint32_t)((draw >> 32) % (c->cfg.noop_max + 1ull));
            nfr[r * K + k] = (uint16_t)(1 + c->cfg.startup_frames + noops);
        }
        for (uint32_t k0 = 0; k0 < K; k0 += kLanes) {
            Tile t;
            std::memset(&t, 0xFF, sizeof(t));
            t.rom = (int32_t)r;
            t.count = (int32_t)std::min<uint32_t>(kLanes, K - k0);
            for (int l = 0; l < t.count; ++l) t.env[l] = t.out[l] = (int32_t)(r * K + k0 + l);
            ctiles.push_back(t);
        }
    }
    Tile* d_ct = nullptr;
    uint16_t* d_nfr = nullptr;
    uint8_t* d_clog = nullptr;
    StepInfo* d_cinfo = nullptr;
    uint32_t* d_cnt = nullptr;
    rc = alloc_n(c, &d_ct, ctiles.size(), "cache tiles");
    if (!rc) rc = alloc_n(c, &d_nfr, M, "cache frame counts");
    if (!rc) rc = alloc_n(c, &d_clog, (size_t)M * 2 * kFrameLogBytes, "cache row logs");
    if (!rc) rc = alloc_n(c, &d_cinfo, M, "cache info");
    if (!rc) rc = alloc_n(c, &d_cnt, 1, "cache tile count");
    auto cleanup = [&]() {
        dev_free(c, d_ct, ctiles.size() * sizeof(Tile));
        dev_free(c, d_nfr, (size_t)M * 2);
        dev_free(c, d_clog, (size_t)M * 2 * kFrameLogBytes);
        dev_free(c, d_cinfo, (size_t)M * sizeof(StepInfo));
        dev_free(c, d_cnt, 4);
    };
    if (rc) {
        cleanup();
        return rc;
    }
    const uint32_t n_ct = (uint32_t)ctiles.size();
    if (hipMemcpy(d_ct, ctiles.data(), ctiles.size() * sizeof(Tile), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d_nfr, nfr.data(), (size_t)M * 2, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d_cnt, &n_ct, 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_cache_state, cst.data(), (size_t)M * sizeof(DevEnv), hipMemcpyHostToDevice) != hipSuccess) {
        cleanup();
        return fail(VCS_E_HIP, "cache upload failed");
    }
    InterpArgs ia{};
    ia.tiles = d_ct;
    ia.n_tiles = d_cnt;
    ia.envs = c->d_cache_state;
    ia.roms = c->d_roms;
    ia.schemes = c->d_schemes;
    ia.actions = nullptr;
    ia.nframes_per_out = d_nfr;
    ia.nframes = 0;
    ia.render_all = 0;
    ia.log_enabled = 1;
    ia.early_stop = 0;
    ia.sticky_thr = 0;
    ia.frameskip = 1;
    ia.seed = c->cfg.seed;
    ia.logs = d_clog;
    ia.n_slots = 2;
    ia.info = d_cinfo;
    ia.reward = nullptr;
    ia.done = nullptr;
    ia.err_word = c->d_err;
    ia.instr_total = nullptr;
    launch_interp(ia, n_ct, nullptr);
    RenderArgs ra{};
    ra.logs = d_clog;
    ra.n_slots = 2;
    ra.info = d_cinfo;
    ra.frames = nullptr;
    ra.obs = c->d_cache_obs;
    ra.gray = c->d_gray;
    ra.n = M;
    ra.force_obs = 1;
    launch_render_obs(ra, nullptr);
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipDeviceSynchronize();
    std::vector<StepInfo> cinfo(M);
    hipError_t e3 = hipMemcpy(cinfo.data(), d_cinfo, (size_t)M * sizeof(StepInfo), hipMemcpyDeviceToHost);
    cleanup();
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess)
        return fail(VCS_E_HIP, std::string("cache build failed: ") + hipGetErrorString(e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e3)));
    for (uint32_t i = 0; i < M; ++i)
        if (cinfo[i].err)
            return fail(VCS_E_ROM, "ROM " + std::to_string(i / K) + " faults while building its reset cache (error bits " +
                                       std::to_string(cinfo[i].err) + ")");
    // clear the bookkeeping the build left in the entries
    HIP_OK(hipMemcpy(cst.data(), c->d_cache_state, (size_t)M * sizeof(DevEnv), hipMemcpyDeviceToHost));
    for (auto& e : cst) {
        e.step_idx = 0;
        e.episode_idx = 0;
        e.prev_action = 0;
        e.err = 0;
    }
    HIP_OK(hipMemcpy(c->d_cache_state, cst.data(), (size_t)M * sizeof(DevEnv), hipMemcpyHostToDevice));

    // ---- every env starts from a cache entry (episode 0)
    std::vector<DevEnv> envs(N);
    for (uint32_t e = 0; e < N; ++e) {
        std::memset(&envs[e], 0, sizeof(DevEnv));
        envs[e].rom_id = env_rom_host[e];
    }
    HIP_OK(hipMemcpy(c->d_envs, envs.data(), (size_t)N * sizeof(DevEnv), hipMemcpyHostToDevice));
    ResetArgs rs{};
    rs.envs = c->d_envs;
    rs.ids = nullptr;
    rs.n = N;
    rs.num_envs = N;
    rs.info = nullptr;
    rs.valid = nullptr;
    rs.cache_state = c->d_cache_state;
    rs.cache_obs = c->d_cache_obs;
    rs.K = K;
    rs.seed = c->cfg.seed;
    rs.obs = nullptr;
    launch_reset(rs, nullptr);
    HIP_OK(hipGetLastError());
    HIP_OK(hipDeviceSynchronize());
    HIP_OK(hipMemset(c->d_err, 0, 4));
    HIP_OK(hipMemset(c->d_err + 1, 0xFF, 4));
    c->assigned = true;
    return VCS_OK;
}

int vcs_reset(vcs_ctx* c, const int32_t* ids, uint32_t n, uint8_t* obs, void* stream) {
    if (!c) return fail(VCS_E_INVAL, "null context");
    if (!c->assigned) return fail(VCS_E_STATE, "vcs_assign first");
    if (n > c->max_batch) return fail(VCS_E_INVAL, "n exceeds max_batch");
    if (n == 0) return VCS_OK;
    hipStream_t s = (hipStream_t)stream;
    ResetArgs rs{};
    rs.envs = c->d_envs;
    rs.ids = ids;
    rs.n = n;
    rs.num_envs = c->cfg.num_envs;
    rs.info = nullptr;
    rs.valid = nullptr;
    if (ids) {
        launch_fill_u32(c->d_counts, c->n_roms, 0, s);
        launch_validate(ids, n, c->cfg.num_envs, c->d_env_rom, c->d_claim, c->tag++, c->d_counts, c->d_valid,
                        nullptr, nullptr, nullptr, c->d_err, s);
        rs.valid = c->d_valid;
    }
    rs.cache_state = c->d_cache_state;
    rs.cache_obs = c->d_cache_obs;
    rs.K = c->cfg.reset_cache_k;
    rs.seed = c->cfg.seed;
    rs.obs = obs;
    begin_timed(c, 3, s);
    launch_reset(rs, s);
    end_timed(c, s);
    HIP_OK(hipGetLastError());
    return VCS_OK;
}

int vcs_step(vcs_ctx* c, const int32_t* ids, const uint8_t* actions, uint32_t n, uint8_t* obs, int32_t* reward,
             uint8_t* done, uint8_t* frames, void* stream) {
    if (!c) return fail(VCS_E_INVAL, "null context");
    if (!c->assigned) return fail(VCS_E_STATE, "vcs_assign first");
    if (n > c->max_batch) return fail(VCS_E_INVAL, "n exceeds max_batch");
    if (n == 0) return VCS_OK;
    if (!actions || !reward || !done) return fail(VCS_E_INVAL, "actions, reward and done are required");
    hipStream_t s = (hipStream_t)stream;
    const Tile* tiles = c->d_tiles_all;
    const uint32_t* n_tiles = c->d_n_tiles_all;
    uint32_t grid = c->n_tiles_all;
    if (ids || n != c->cfg.num_envs) {
        int rc = build_tiles(c, ids, n, reward, done, s, &grid);
        if (rc) return rc;
        tiles = c->d_tiles;
        n_tiles = c->d_n_tiles;
    }
    launch_fill_u32(reinterpret_cast<uint32_t*>(c->d_instr), 4, 0, s);
    InterpArgs ia{};
    ia.tiles = tiles;
    ia.n_tiles = n_tiles;
    ia.envs = c->d_envs;
    ia.roms = c->d_roms;
    ia.schemes = c->d_schemes;
    ia.actions = actions;
    ia.nframes_per_out = nullptr;
    ia.nframes = c->cfg.frameskip;
    ia.render_all = c->cfg.render_mode == VCS_RENDER_ALL;
    ia.log_enabled = (obs || frames) ? 1 : 0;
    ia.early_stop = 1;
    ia.sticky_thr = c->cfg.sticky_threshold;
    ia.frameskip = c->cfg.frameskip;
    ia.seed = c->cfg.seed;
    ia.logs = c->d_logs;
    ia.n_slots = c->n_slots;
    ia.info = c->d_info;
    ia.reward = reward;
    ia.done = done;
    ia.err_word = c->d_err;
    ia.instr_total = c->d_instr;
    begin_timed(c, 0, s);
    launch_interp(ia, grid, s);
    end_timed(c, s);

    RenderArgs ra{};
    ra.logs = c->d_logs;
    ra.n_slots = c->n_slots;
    ra.info = c->d_info;
    ra.frames = frames;
    ra.obs = obs;
    ra.gray = c->d_gray;
    ra.n = n;
    ra.force_obs = 0;
    if (frames && c->n_slots > 2) {
        begin_timed(c, 1, s);
        launch_render_frames(ra, c->n_slots - 2, s);
        end_timed(c, s);
    }
    if (obs || frames) {
        begin_timed(c, 2, s);
        launch_render_obs(ra, s);
        end_timed(c, s);
    }
    ResetArgs rs{};
    rs.envs = c->d_envs;
    rs.ids = ids;
    rs.n = n;
    rs.num_envs = c->cfg.num_envs;
    rs.info = c->d_info;
    rs.valid = nullptr;
    rs.cache_state = c->d_cache_state;
    rs.cache_obs = c->d_cache_obs;
    rs.K = c->cfg.reset_cache_k;
    rs.seed = c->cfg.seed;
    rs.obs = obs;
    begin_timed(c, 3, s);
    launch_reset(rs, s);
    end_timed(c, s);
    HIP_OK(hipGetLastError());
    return VCS_OK;
}

int vcs_get_state(vcs_ctx* c, uint32_t env, uint8_t* out) {
    if (!c || !out) return fail(VCS_E_INVAL, "null argument");
    if (env >= c->cfg.num_envs) return fail(VCS_E_INVAL, "env id out of range");
    HIP_OK(hipSetDevice(c->cfg.device));
    HIP_OK(hipDeviceSynchronize());
    DevEnv e;
    HIP_OK(hipMemcpy(&e, c->d_envs + env, sizeof(DevEnv), hipMemcpyDeviceToHost));
    to_record(e, out);
    return VCS_OK;
}

int vcs_set_state(vcs_ctx* c, uint32_t env, const uint8_t* in) {
    if (!c || !in) return fail(VCS_E_INVAL, "null argument");
    if (env >= c->cfg.num_envs) return fail(VCS_E_INVAL, "env id out of range");
    if (!c->assigned) return fail(VCS_E_STATE, "vcs_assign first");
    DevEnv e;
    if (from_record(in, &e)) return fail(VCS_E_INVAL, "bad timer fields in state record");
    if (e.rom_id >= c->n_roms) return fail(VCS_E_INVAL, "state names an unknown ROM");
    if (e.rom_id != c->h_env_rom[env]) return fail(VCS_E_INVAL, "state's ROM differs from the env's ROM");
    if (c->h_schemes[e.rom_id] == VCS_BANK_4K && e.bank != 0) return fail(VCS_E_INVAL, "bank must be 0 for a 4K ROM");
    if (e.bank > 1) return fail(VCS_E_INVAL, "bank must be 0 or 1");
    HIP_OK(hipSetDevice(c->cfg.device));
    HIP_OK(hipDeviceSynchronize());
    HIP_OK(hipMemcpy(c->d_envs + env, &e, sizeof(DevEnv), hipMemcpyHostToDevice));
    return VCS_OK;
}

int vcs_get_cache(vcs_ctx* c, uint32_t rom, uint32_t k, uint8_t* state, uint8_t* obs) {
    if (!c) return fail(VCS_E_INVAL, "null context");
    if (!c->assigned || rom >= c->n_roms || k >= c->cfg.reset_cache_k) return fail(VCS_E_INVAL, "no such cache entry");
    HIP_OK(hipSetDevice(c->cfg.device));
    HIP_OK(hipDeviceSynchronize());
    const size_t idx = (size_t)rom * c->cfg.reset_cache_k + k;
    if (state) {
        DevEnv e;
        HIP_OK(hipMemcpy(&e, c->d_cache_state + idx, sizeof(DevEnv), hipMemcpyDeviceToHost));
        to_record(e, state);
    }
    if (obs) HIP_OK(hipMemcpy(obs, c->d_cache_obs + idx * kObsBytes, kObsBytes, hipMemcpyDeviceToHost));
    return VCS_OK;
}

int vcs_poll_errors(vcs_ctx* c, uint32_t* first_env, uint32_t* bits) {
    if (!c || !first_env || !bits) return fail(VCS_E_INVAL, "null argument");
    HIP_OK(hipSetDevice(c->cfg.device));
    HIP_OK(hipDeviceSynchronize());
    uint32_t w[2];
    HIP_OK(hipMemcpy(w, c->d_err, 8, hipMemcpyDeviceToHost));
    *bits = w[0];
    *first_env = w[1];
    HIP_OK(hipMemset(c->d_err, 0, 4));
    HIP_OK(hipMemset(c->d_err + 1, 0xFF, 4));
    return VCS_OK;
}

int vcs_last_step_instructions(vcs_ctx* c, uint64_t* out) {
    if (!c || !out) return fail(VCS_E_INVAL, "null argument");
    HIP_OK(hipSetDevice(c->cfg.device));
    HIP_OK(hipDeviceSynchronize());
    unsigned long long v = 0;
    HIP_OK(hipMemcpy(&v, c->d_instr, 8, hipMemcpyDeviceToHost));
    *out = v;
    return VCS_OK;
}

int vcs_last_step_stats(vcs_ctx* c, uint64_t* out2) {
    if (!c || !out2) return fail(VCS_E_INVAL, "null argument");
    HIP_OK(hipSetDevice(c->cfg.device));
    HIP_OK(hipDeviceSynchronize());
    unsigned long long v[2] = {0, 0};
    HIP_OK(hipMemcpy(v, c->d_instr, 16, hipMemcpyDeviceToHost));
    out2[0] = v[0];
    out2[1] = v[1];
    return VCS_OK;
}

int vcs_timing(vcs_ctx* c, int enable) {
    if (!c) return fail(VCS_E_INVAL, "null context");
    if (enable) clear_timed(c);
    c->timing = enable != 0;
    return VCS_OK;
}

int vcs_kernel_time(vcs_ctx* c, int which, double* mean_ms, uint32_t* launches) {
    if (!c || !mean_ms || !launches) return fail(VCS_E_INVAL, "null argument");
    double total = 0;
    uint32_t cnt = 0;
    for (auto& t : c->timed) {
        if (t.kind != which) continue;
        HIP_OK(hipEventSynchronize(t.stop));
        float ms = 0;
        HIP_OK(hipEventElapsedTime(&ms, t.start, t.stop));
        total += ms;
        ++cnt;
    }
    *mean_ms = cnt ? total / cnt : 0.0;
    *launches = cnt;
    return VCS_OK;
}

}  // extern "C"
