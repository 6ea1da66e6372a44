// vcs355 C ABI: context, device memory plan and the step/reset pipelines.
//
// Per step (all on the caller's stream, no host synchronisation):
//   k_step_begin       clear the per-call counters (and the tile queue)
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

// Scratch of one step pipeline.  d_stepw holds the per-call words
// [counts R][offsets R][fill R] (pad) [instruction counters, 2 x u64][queue].
struct Pipe {
    uint8_t* d_logs = nullptr;      // [max_batch][n_slots] row logs
    uint8_t* d_cxlogs = nullptr;    // [max_batch] logs of unrendered frames (tracked collisions)
    uint16_t* d_nfpo = nullptr;     // [max_batch] no-ops after the copy: frames each reset env runs
    uint8_t* d_nooplogs = nullptr;  // [max_batch][2] row logs of those frames' last two
    StepInfo* d_noopinfo = nullptr; // [max_batch]
    StepInfo* d_info = nullptr;     // [max_batch]
    uint8_t* d_valid = nullptr;     // [max_batch]
    Tile* d_tiles = nullptr;        // [tiles_cap]
    uint32_t* d_n_tiles = nullptr;
    uint32_t* d_tag = nullptr;      // claim tag: residue + 16 x (calls that validated ids)
    uint32_t residue = 0;           // its tags' residue mod 16: the pipeline index (8: the shared scratch)
    uint32_t* d_stepw = nullptr;
    uint32_t* d_counts = nullptr;
    unsigned long long* d_instr = nullptr;
    uint32_t* d_queue = nullptr;
};

struct vcs_ctx {
    vcs_config cfg{};
    uint32_t max_batch = 0;
    uint32_t n_slots = 0;
    size_t allocated = 0;
    std::vector<void*> owned;

    // ROMs
    uint32_t n_roms = 0;
    uint8_t* d_roms = nullptr;
    uint32_t* d_pre = nullptr;
    size_t pre_words = 0;
    CartMap* d_cmap = nullptr;
    uint32_t* d_pre_off = nullptr;
    std::vector<uint32_t> h_schemes;
    std::vector<RomInfo> h_rinfo;
    std::vector<uint8_t> h_roms;   // [n_roms][kRomSlot]
    uint32_t rom_lds = 8192;       // cartridge bytes the interpreter stages in LDS (0: reads HBM)

    // envs
    DevEnv* d_envs = nullptr;
    uint16_t* d_env_rom = nullptr;
    std::vector<uint16_t> h_env_rom;
    bool assigned = false;

    // reset cache
    DevEnv* d_cache_state = nullptr;
    uint8_t* d_cache_obs = nullptr;

    // launch shape and tiles
    vcs_launch launch{64, 0, 256};
    uint32_t n_cu = 0;
    uint64_t generation = 0;        // bumped when tiles or the launch shape change
    Tile* d_tiles_all = nullptr;
    uint32_t n_tiles_all = 0;
    uint32_t* d_n_tiles_all = nullptr;
    uint32_t* d_claim = nullptr;
    uint32_t stepw_words = 0;
    uint32_t instr_off = 0;         // word offset of the instruction counters in Pipe::d_stepw
    uint32_t tiles_cap = 0;         // tiles per pipeline buffer

    // per-pipeline scratch: calls on different pipelines may run concurrently
    std::vector<Pipe> pipes;

    uint32_t* d_err = nullptr;
    uint8_t* d_gray = nullptr;

    // timing
    bool timing = false;
    std::vector<TimedLaunch> timed;
};

// ---------------------------------------------------------------- static scratch
//
// The scratch of vcs_step_noalloc: row logs for the last two frames of up to
// kNoAllocEnvs envs, the logs of unrendered frames for tracked collisions,
// step info, id validity, tiles, per-call counters and a claim tag, in one
// file-scope device array.  Every GPU the library runs on holds its own copy
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress gives on that device (g_scratch, taken when a context
// is created there).  All calls on one GPU share it.
constexpr uint32_t kNoAllocEnvs = 512;
constexpr uint32_t kNoAllocRoms = 1024;
constexpr uint32_t kNoAllocTiles = kNoAllocEnvs + kNoAllocRoms;    // tiles of 1 env each, + one partial per ROM
constexpr uint32_t kNoAllocStepw = 3 * kNoAllocRoms + 16;         // per-call words of kNoAllocRoms ROMs
constexpr size_t sc_align(size_t b) { return (b + 255) & ~size_t(255); }
constexpr size_t kScLogs = 0;
constexpr size_t kScCxLogs = kScLogs + sc_align((size_t)kNoAllocEnvs * 2 * kFrameLogBytes);
constexpr size_t kScInfo = kScCxLogs + sc_align((size_t)kNoAllocEnvs * kFrameLogBytes);
constexpr size_t kScValid = kScInfo + sc_align(kNoAllocEnvs * sizeof(StepInfo));
constexpr size_t kScTiles = kScValid + sc_align(kNoAllocEnvs);
constexpr size_t kScNTiles = kScTiles + sc_align((size_t)kNoAllocTiles * sizeof(Tile));
constexpr size_t kScTag = kScNTiles + 256;
constexpr size_t kScStepw = kScTag + 256;
constexpr size_t kScratchBytes = kScStepw + sc_align(kNoAllocStepw * 4);   // 43.7 MB
constexpr uint32_t kScratchResidue = 8;   // claim tags of the shared scratch: 8 mod 16
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {

uint8_t* g_scratch[kMaxDevices] = {};   // scratch's address on each device (nullptr: not taken yet)

// Take scratch's device address on `dev` (current) once; the array's host
// name is no device address.
int take_scratch_address(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return fail(VCS_E_INVAL, "device ordinal beyond the scratch table");
    if (g_scratch[dev]) return VCS_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(VCS_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = static_cast<uint8_t*>(ptr);
    return VCS_OK;
}

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
    const RomInfo& R = c->h_rinfo[r];
    // power-on bank: the last 4 KB bank; E0 slices 4, 5, 6; 3F slice 0
    const uint32_t bank = R.kind == CART_E0 ? (4u | (5u << 3) | (6u << 6)) : R.kind == CART_3F ? 0u : R.n_vbanks - 1;
    e.sp = 0xFD;
    e.p = 0x24;
    e.bank = (uint8_t)bank;
    e.bank_hi = (uint8_t)(bank >> 8);
    e.track_cx = c->cfg.collisions ? 1 : 0;
    e.pc = (uint16_t)(rom[cart_rom_off(R, bank, 0x1FFC)] | (rom[cart_rom_off(R, bank, 0x1FFD)] << 8));
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
    out[31] = e.bank_hi;
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
    const uint8_t* t2 = e.tia2;   // R[16..47]
    auto R = [&](int i) { return t2[i - 16]; };
    const uint8_t objs[19] = {R(R_NUSIZ0), R(R_NUSIZ1), R(R_ENAM0), R(R_ENAM1), R(R_ENABL), R(R_ENABL_OLD),
                              R(R_GRP0_OLD), R(R_GRP1_OLD), R(R_VDELP0), R(R_VDELP1), R(R_VDELBL), R(R_RESMP0),
                              R(R_RESMP1), R(R_M0X), R(R_M1X), R(R_BLX), R(R_HMM0), R(R_HMM1), R(R_HMBL)};
    std::memcpy(out + 208, objs, 19);
    out[227] = e.hmb_now;
    std::memcpy(out + 228, &e.cx, 2);
    out[230] = e.track_cx;
    std::memcpy(out + 256, e.xram, 128);
}

int from_record(const uint8_t* in, DevEnv* e) {
    std::memset(e, 0, sizeof(*e));
    e->a = in[0]; e->x = in[1]; e->y = in[2]; e->sp = in[3]; e->p = in[4]; e->bank = in[5];
    e->bank_hi = in[31];
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
    const uint8_t* o = in + 208;
    uint8_t* t2 = e->tia2;
    auto W = [&](int i, uint8_t v) { t2[i - 16] = v; };
    W(R_NUSIZ0, o[0]); W(R_NUSIZ1, o[1]); W(R_ENAM0, o[2]); W(R_ENAM1, o[3]); W(R_ENABL, o[4]);
    W(R_ENABL_OLD, o[5]); W(R_GRP0_OLD, o[6]); W(R_GRP1_OLD, o[7]); W(R_VDELP0, o[8]); W(R_VDELP1, o[9]);
    W(R_VDELBL, o[10]); W(R_RESMP0, o[11]); W(R_RESMP1, o[12]); W(R_M0X, o[13]); W(R_M1X, o[14]);
    W(R_BLX, o[15]); W(R_HMM0, o[16]); W(R_HMM1, o[17]); W(R_HMBL, o[18]);
    // the renderer's flag bits: ENAM0, ENAM1, ENABL, ENABL (delayed), RESMP0 D1; VDELP0, VDELP1, VDELBL D0
    const uint8_t flags = (uint8_t)(((o[2] >> 1) & 1) | (((o[3] >> 1) & 1) << 1) | (((o[4] >> 1) & 1) << 2) |
                                    (((o[5] >> 1) & 1) << 3) | ((o[8] & 1) << 4) | ((o[9] & 1) << 5) |
                                    ((o[10] & 1) << 6) | (((o[11] >> 1) & 1) << 7));
    W(R_FLAGS, flags);
    W(R_FLAGS2, (uint8_t)((o[12] >> 1) & 1));
    e->hmb_now = in[227] ? 1 : 0;
    if (e->hmb_now) {   // the blanked line may be a row of the current frame
        const int64_t row = (int64_t)(e->cycle / 76) - (int64_t)e->frame_line0 - kFirstRow;
        if (row >= 0 && row < kRows) W(R_HMB, (uint8_t)(row + 1));
    }
    std::memcpy(&e->cx, in + 228, 2);
    e->track_cx = in[230] ? 1 : 0;
    std::memcpy(e->xram, in + 256, 128);
    return 0;
}

// Build ROM-homogeneous tiles on the device for the ids of one call.  The
// counters were cleared and the claim tag advanced by k_step_begin.
int build_tiles(vcs_ctx* c, Pipe& P, const int32_t* ids, uint32_t n, int32_t* reward, uint8_t* done, hipStream_t s,
                uint32_t* grid) {
    const uint32_t R = c->n_roms, w = c->launch.tile_envs;
    uint32_t* counts = P.d_counts;
    uint32_t* offsets = P.d_counts + R;
    uint32_t* fill = P.d_counts + 2 * R;
    launch_validate(ids, n, c->cfg.num_envs, c->d_env_rom, c->d_claim, P.d_tag, counts, P.d_valid, P.d_info,
                    reward, done, c->d_err, s);
    launch_tile_layout(counts, R, w, offsets, fill, P.d_tiles, P.d_n_tiles, s);
    launch_tile_fill(ids, n, c->d_env_rom, P.d_valid, w, offsets, fill, P.d_tiles, s);
    *grid = (n + w - 1) / w + R;
    HIP_OK(hipGetLastError());
    return VCS_OK;
}

// (Re)allocate the per-call tile buffers for the current ROM count and width.
int ensure_tile_buffer(vcs_ctx* c) {
    const uint32_t cap = (c->max_batch + c->launch.tile_envs - 1) / c->launch.tile_envs + c->n_roms;
    bool have = c->tiles_cap >= cap && c->tiles_cap / 4 <= cap;
    for (auto& P : c->pipes) have = have && P.d_tiles;
    if (have) return VCS_OK;
    for (auto& P : c->pipes) {
        dev_free(c, P.d_tiles, (size_t)c->tiles_cap * sizeof(Tile));
        P.d_tiles = nullptr;
    }
    c->tiles_cap = 0;
    for (auto& P : c->pipes) {
        int rc = alloc_n(c, &P.d_tiles, cap, "tiles");
        if (rc) return rc;
    }
    c->tiles_cap = cap;
    return VCS_OK;
}

// Tiles over all envs, ROM by ROM, `tile_envs` envs each (env id = output position).
int build_all_tiles(vcs_ctx* c) {
    const uint32_t N = c->cfg.num_envs, R = c->n_roms, w = c->launch.tile_envs;
    std::vector<Tile> tiles;
    std::vector<std::vector<int32_t>> by_rom(R);
    for (uint32_t e = 0; e < N; ++e) by_rom[c->h_env_rom[e]].push_back((int32_t)e);
    for (uint32_t r = 0; r < R; ++r) {
        for (size_t i = 0; i < by_rom[r].size(); i += w) {
            Tile t;
            std::memset(&t, 0xFF, sizeof(t));
            t.rom = (int32_t)r;
            t.count = (int32_t)std::min<size_t>(w, by_rom[r].size() - i);
            for (int l = 0; l < t.count; ++l) t.env[l] = t.out[l] = by_rom[r][i + l];
            tiles.push_back(t);
        }
    }
    dev_free(c, c->d_tiles_all, (size_t)c->n_tiles_all * sizeof(Tile));
    c->d_tiles_all = nullptr;
    c->n_tiles_all = 0;
    int rc = alloc_n(c, &c->d_tiles_all, tiles.size(), "tiles (all envs)");
    if (rc) return rc;
    c->n_tiles_all = (uint32_t)tiles.size();
    HIP_OK(hipMemcpy(c->d_tiles_all, tiles.data(), tiles.size() * sizeof(Tile), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(c->d_n_tiles_all, &c->n_tiles_all, 4, hipMemcpyHostToDevice));
    return VCS_OK;
}

bool pow2_le64(uint32_t w) { return w >= 1 && w <= 64 && (w & (w - 1)) == 0; }

int check_launch(const vcs_launch* l) {
    if (!pow2_le64(l->tile_envs)) return fail(VCS_E_INVAL, "tile_envs must be a power of two in [1, 64]");
    if (l->workers > (1u << 20)) return fail(VCS_E_INVAL, "workers must be <= 2^20");
    const uint32_t b = l->render_block;
    if (b != 64 && b != 128 && b != 256 && b != 512) return fail(VCS_E_INVAL, "render_block must be 64, 128, 256 or 512");
    return VCS_OK;
}

// No-ops after the copy: the envs k_reset just restarted (P.d_nfpo[i] > 0)
// run their 2 + n NOOP frames over the same tiles (the others run none),
// logging the last two, whose observation then goes to obs[i] for those
// positions only.  The step counter does not advance.
static int enqueue_noops(vcs_ctx* c, Pipe& P, const Tile* tiles, const uint32_t* n_tiles, uint32_t grid,
                         uint32_t n, uint8_t* obs, hipStream_t s) {
    InterpArgs ia{};
    ia.tiles = tiles;
    ia.n_tiles = n_tiles;
    ia.envs = c->d_envs;
    ia.roms = c->d_roms;
    ia.cmap = c->d_cmap;
    ia.pre_off = c->d_pre_off;
    ia.pre = c->d_pre;
    ia.actions = nullptr;
    ia.nframes_per_out = P.d_nfpo;
    ia.nframes = 0;
    ia.render_all = 0;
    ia.log_enabled = obs ? 1 : 0;
    ia.early_stop = 0;
    ia.sticky_thr = 0;
    ia.frameskip = c->cfg.frameskip;
    ia.seed = c->cfg.seed;
    ia.logs = P.d_nooplogs;
    ia.n_slots = 2;
    ia.info = P.d_noopinfo;
    ia.reward = nullptr;
    ia.done = nullptr;
    ia.err_word = c->d_err;
    ia.instr_total = P.d_instr;
    ia.queue = nullptr;
    ia.track = c->cfg.collisions ? 1 : 0;
    ia.cx_logs = P.d_cxlogs;
    ia.count_step = 0;
    launch_interp(ia, grid, c->launch.tile_envs, c->rom_lds, s);
    if (obs) {
        RenderArgs ra{};
        ra.logs = P.d_nooplogs;
        ra.n_slots = 2;
        ra.info = P.d_noopinfo;
        ra.frames = nullptr;
        ra.obs = obs;
        ra.gray = c->d_gray;
        ra.n = n;
        ra.force_obs = 1;
        ra.only = P.d_nfpo;
        launch_render_obs(ra, c->launch.render_block, s);
    }
    HIP_OK(hipGetLastError());
    return VCS_OK;
}

// The emulation part of one step on stream s with the scratch of pipeline
// `pipe` (arguments checked): counters, id validation and tiles, the
// interpreter (frames, row logs, reward, done) and the eager reset.
// P: the scratch (a pipeline's, or the shared static one); n_slots / render_all:
// the frame slots its row logs hold and whether every frame is logged (the
// context's render mode, or 2 and the last two frames).
int enqueue_sim_on(vcs_ctx* c, Pipe& P, uint32_t n_slots, bool render_all, const int32_t* ids,
                   const uint8_t* actions, uint32_t n, uint8_t* obs, int32_t* reward, uint8_t* done, uint8_t* frames,
                   hipStream_t s) {
    const Tile* tiles = c->d_tiles_all;
    const uint32_t* n_tiles = c->d_n_tiles_all;
    uint32_t grid = c->n_tiles_all;
    const bool listed = ids || n != c->cfg.num_envs;
    if (listed) {
        // counts, offsets, fill, instruction counters and queue; advance the tag
        launch_step_begin(P.d_stepw, c->stepw_words, P.d_tag, P.residue, s);
        int rc = build_tiles(c, P, ids, n, reward, done, s, &grid);
        if (rc) return rc;
        tiles = P.d_tiles;
        n_tiles = P.d_n_tiles;
    } else {
        launch_step_begin(P.d_stepw + c->instr_off, c->stepw_words - c->instr_off, nullptr, 0, s);
    }
    InterpArgs ia{};
    ia.tiles = tiles;
    ia.n_tiles = n_tiles;
    ia.envs = c->d_envs;
    ia.roms = c->d_roms;
    ia.cmap = c->d_cmap;
    ia.pre_off = c->d_pre_off;
    ia.pre = c->d_pre;
    ia.actions = actions;
    ia.nframes_per_out = nullptr;
    ia.nframes = c->cfg.frameskip;
    ia.render_all = render_all ? 1 : 0;
    ia.log_enabled = (obs || frames) ? 1 : 0;
    ia.early_stop = 1;
    ia.sticky_thr = c->cfg.sticky_threshold;
    ia.frameskip = c->cfg.frameskip;
    ia.seed = c->cfg.seed;
    ia.logs = P.d_logs;
    ia.n_slots = n_slots;
    ia.info = P.d_info;
    ia.reward = reward;
    ia.done = done;
    ia.err_word = c->d_err;
    ia.instr_total = P.d_instr;
    ia.queue = nullptr;
    ia.track = c->cfg.collisions ? 1 : 0;
    ia.cx_logs = P.d_cxlogs;
    ia.count_step = 1;
    const uint32_t full_grid = grid;
    if (c->launch.workers && c->launch.workers < grid) {
        ia.queue = P.d_queue;
        grid = c->launch.workers;
    }
    begin_timed(c, 0, s);
    launch_interp(ia, grid, c->launch.tile_envs, c->rom_lds, s);
    end_timed(c, s);

    // a done env restarts from the cache now (state, and its observation);
    // the render below leaves done envs' observations alone
    ResetArgs rs{};
    rs.envs = c->d_envs;
    rs.ids = ids;
    rs.n = n;
    rs.num_envs = c->cfg.num_envs;
    rs.info = P.d_info;
    rs.valid = nullptr;
    rs.cache_state = c->d_cache_state;
    rs.cache_obs = c->d_cache_obs;
    rs.K = c->cfg.reset_cache_k;
    rs.seed = c->cfg.seed;
    rs.obs = obs;
    rs.nfpo = c->cfg.noop_after_copy ? P.d_nfpo : nullptr;
    rs.noop_max = c->cfg.noop_max;
    begin_timed(c, 3, s);
    launch_reset(rs, s);
    end_timed(c, s);
    HIP_OK(hipGetLastError());
    if (c->cfg.noop_after_copy) return enqueue_noops(c, P, tiles, n_tiles, full_grid, n, obs, s);
    return VCS_OK;
}

int enqueue_sim(vcs_ctx* c, uint32_t pipe, const int32_t* ids, const uint8_t* actions, uint32_t n, uint8_t* obs,
                int32_t* reward, uint8_t* done, uint8_t* frames, hipStream_t s) {
    return enqueue_sim_on(c, c->pipes[pipe], c->n_slots, c->cfg.render_mode == VCS_RENDER_ALL, ids, actions, n, obs,
                          reward, done, frames, s);
}

// Render of one step from pipeline `pipe`'s row logs: frames output and
// observations.  Needs only that step's interpreter launch; the env state is
// not touched, so it may overlap the next step's interpreter on another
// pipeline.
int enqueue_render_on(vcs_ctx* c, Pipe& P, uint32_t n_slots, uint32_t n, uint8_t* obs, uint8_t* frames,
                      hipStream_t s) {
    RenderArgs ra{};
    ra.logs = P.d_logs;
    ra.n_slots = n_slots;
    ra.info = P.d_info;
    ra.frames = frames;
    ra.obs = obs;
    ra.gray = c->d_gray;
    ra.n = n;
    ra.force_obs = 0;
    if (frames && n_slots > 2) {
        begin_timed(c, 1, s);
        launch_render_frames(ra, n_slots - 2, c->launch.render_block, s);
        end_timed(c, s);
    }
    if (obs || frames) {
        begin_timed(c, 2, s);
        launch_render_obs(ra, c->launch.render_block, s);
        end_timed(c, s);
    }
    HIP_OK(hipGetLastError());
    return VCS_OK;
}

int enqueue_render(vcs_ctx* c, uint32_t pipe, uint32_t n, uint8_t* obs, uint8_t* frames, hipStream_t s) {
    return enqueue_render_on(c, c->pipes[pipe], c->n_slots, n, obs, frames, s);
}

// One whole step on stream s.
int enqueue_step(vcs_ctx* c, uint32_t pipe, const int32_t* ids, const uint8_t* actions, uint32_t n, uint8_t* obs,
                 int32_t* reward, uint8_t* done, uint8_t* frames, hipStream_t s) {
    int rc = enqueue_sim(c, pipe, ids, actions, n, obs, reward, done, frames, s);
    if (!rc) rc = enqueue_render(c, pipe, n, obs, frames, s);
    return rc;
}

int check_step_args(vcs_ctx* c, uint32_t n, const uint8_t* actions, const int32_t* reward, const uint8_t* done) {
    if (!c) return fail(VCS_E_INVAL, "null context");
    if (!c->assigned) return fail(VCS_E_STATE, "vcs_assign first");
    if (n > c->max_batch) return fail(VCS_E_INVAL, "n exceeds max_batch");
    if (n == 0) return VCS_OK;
    if (!actions || !reward || !done) return fail(VCS_E_INVAL, "actions, reward and done are required");
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
    if (cfg->pipelines > 8) return fail(VCS_E_INVAL, "pipelines must be in [0, 8]");
    if (cfg->noop_after_copy > 1) return fail(VCS_E_INVAL, "noop_after_copy must be 0 or 1");
    if (cfg->noop_after_copy && cfg->startup_frames < 2)
        return fail(VCS_E_INVAL, "noop_after_copy needs startup_frames >= 2");
    int ndev = 0;
    HIP_OK(hipGetDeviceCount(&ndev));
    if (cfg->device < 0 || cfg->device >= ndev) return fail(VCS_E_INVAL, "bad device ordinal");
    HIP_OK(hipSetDevice(cfg->device));

    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, cfg->device));
    vcs_ctx* c = new vcs_ctx();
    c->cfg = *cfg;
    c->n_cu = (uint32_t)prop.multiProcessorCount;
    c->max_batch = cfg->max_batch ? cfg->max_batch : cfg->num_envs;
    c->n_slots = cfg->render_mode == VCS_RENDER_ALL ? cfg->frameskip : 2;
    int rc = VCS_OK;
    const size_t B = c->max_batch;
    if (!rc) rc = alloc_n(c, &c->d_envs, cfg->num_envs, "env state");
    if (!rc) rc = alloc_n(c, &c->d_env_rom, cfg->num_envs, "env rom");
    if (!rc) rc = alloc_n(c, &c->d_claim, cfg->num_envs, "id claims");
    if (!rc) rc = alloc_n(c, &c->d_err, 2, "error word");
    if (!rc) rc = alloc_n(c, &c->d_gray, 128, "gray table");
    if (!rc) rc = alloc_n(c, &c->d_n_tiles_all, 1, "tile count");
    c->pipes.resize(cfg->pipelines ? cfg->pipelines : 1);
    for (auto& P : c->pipes) {
        if (!rc) rc = alloc_n(c, &P.d_logs, B * c->n_slots * kFrameLogBytes, "row logs");
        if (!rc && cfg->collisions) rc = alloc_n(c, &P.d_cxlogs, B * kFrameLogBytes, "collision row logs");
        if (!rc && cfg->noop_after_copy) rc = alloc_n(c, &P.d_nfpo, B, "reset no-op frame counts");
        if (!rc && cfg->noop_after_copy) rc = alloc_n(c, &P.d_nooplogs, B * 2 * kFrameLogBytes, "reset no-op row logs");
        if (!rc && cfg->noop_after_copy) rc = alloc_n(c, &P.d_noopinfo, B, "reset no-op info");
        if (!rc) rc = alloc_n(c, &P.d_info, B, "step info");
        if (!rc) rc = alloc_n(c, &P.d_valid, B, "id validity");
        if (!rc) rc = alloc_n(c, &P.d_tag, 1, "claim tag");
        if (!rc) rc = alloc_n(c, &P.d_n_tiles, 1, "tile count");
    }
    if (rc) {
        vcs_destroy(c);
        return rc;
    }
    bool ok = hipMemcpy(c->d_gray, cfg->gray_lut, 128, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemset(c->d_claim, 0xFF, (size_t)cfg->num_envs * 4) == hipSuccess &&
              hipMemset(c->d_err, 0, 4) == hipSuccess && hipMemset(c->d_err + 1, 0xFF, 4) == hipSuccess &&
              hipMemset(c->d_envs, 0, (size_t)cfg->num_envs * sizeof(DevEnv)) == hipSuccess;
    for (uint32_t p = 0; p < c->pipes.size() && ok; ++p) {
        c->pipes[p].residue = p;
        ok = hipMemcpy(c->pipes[p].d_tag, &p, 4, hipMemcpyHostToDevice) == hipSuccess;
    }
    if (!ok) {
        vcs_destroy(c);
        return fail(VCS_E_HIP, "initial device copies failed");
    }
    rc = take_scratch_address(cfg->device);   // with the device current
    if (rc) {
        vcs_destroy(c);
        return rc;
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
    std::vector<RomInfo> info(n_roms);
    size_t pre_words = 0;
    uint32_t max_bytes = 0;
    for (uint32_t r = 0; r < n_roms; ++r) {
        if (!rom_host[r]) return fail(VCS_E_INVAL, "null ROM pointer");
        const uint32_t sch = scheme[r], b = rom_bytes[r];
        RomInfo& R = info[r];
        R = RomInfo{};
        bool ok = false;
        if (sch == VCS_BANK_4K) {
            ok = b == 2048 || b == 4096;
            R.kind = CART_LINEAR;
            R.n_vbanks = 1;
        } else if (sch >= VCS_BANK_F8 && sch <= VCS_BANK_F4SC) {
            const uint32_t nb = (sch == VCS_BANK_F8 || sch == VCS_BANK_F8SC) ? 2 : (sch == VCS_BANK_F6 || sch == VCS_BANK_F6SC) ? 4 : 8;
            ok = b == 4096 * nb;
            R.kind = CART_LINEAR;
            R.n_vbanks = nb;
            R.hs_n = nb;
            R.hs_first = nb == 2 ? 0xFF8 : nb == 4 ? 0xFF6 : 0xFF4;
            R.sc = sch >= VCS_BANK_F8SC ? 1 : 0;
        } else if (sch == VCS_BANK_E0) {
            ok = b == 8192;
            R.kind = CART_E0;
            R.n_vbanks = 512;
        } else if (sch == VCS_BANK_3F) {
            ok = b == 4096 || b == 8192 || b == 16384 || b == 32768;
            R.kind = CART_3F;
            R.n_vbanks = b / 2048;
            R.tf_mask = b / 2048 - 1;
            R.tf_last = b - 2048;
        }
        if (!ok)
            return fail(VCS_E_ROM, "ROM " + std::to_string(r) + ": scheme " + std::to_string(sch) + " does not take " +
                                       std::to_string(b) + " bytes");
        R.pre_off = (uint32_t)pre_words;
        pre_words += (size_t)R.n_vbanks * 4096;
        max_bytes = std::max(max_bytes, b);
    }
    HIP_OK(hipSetDevice(c->cfg.device));
    HIP_OK(hipDeviceSynchronize());
    dev_free(c, c->d_roms, (size_t)c->n_roms * kRomSlot + 16);
    dev_free(c, c->d_pre, c->pre_words * sizeof(uint32_t));
    dev_free(c, c->d_cmap, (size_t)c->n_roms * sizeof(CartMap));
    dev_free(c, c->d_pre_off, (size_t)c->n_roms * 4);
    for (auto& P : c->pipes) {
        dev_free(c, P.d_stepw, (size_t)c->stepw_words * 4);
        dev_free(c, P.d_tiles, (size_t)c->tiles_cap * sizeof(Tile));
        P.d_tiles = nullptr;
        P.d_stepw = nullptr; P.d_counts = nullptr; P.d_instr = nullptr; P.d_queue = nullptr;
    }
    c->d_roms = nullptr; c->d_pre = nullptr; c->d_cmap = nullptr; c->d_pre_off = nullptr;
    c->pre_words = 0;
    c->stepw_words = 0;
    c->tiles_cap = 0;
    ++c->generation;
    c->assigned = false;
    c->n_roms = n_roms;
    c->h_roms.assign((size_t)n_roms * kRomSlot, 0);
    c->h_schemes.assign(scheme, scheme + n_roms);
    c->h_rinfo = info;
    c->rom_lds = max_bytes > 8192 ? 0u : 8192u;
    for (uint32_t r = 0; r < n_roms; ++r) {
        uint8_t* dst = c->h_roms.data() + (size_t)r * kRomSlot;
        std::memcpy(dst, rom_host[r], rom_bytes[r]);
        if (rom_bytes[r] == 2048) std::memcpy(dst + 2048, rom_host[r], 2048);   // a 2 KB ROM shows twice
    }
    // 16 bytes past the last slot: the per-lane fetch reads the dword after a
    // bank's last instruction word
    int rc = alloc_n(c, &c->d_roms, (size_t)n_roms * kRomSlot + 16, "ROMs");
    if (!rc) rc = alloc_n(c, &c->d_pre, pre_words, "predecoded ROMs");
    if (!rc) c->pre_words = pre_words;
    if (!rc) rc = alloc_n(c, &c->d_cmap, n_roms, "ROM mappings");
    if (!rc) rc = alloc_n(c, &c->d_pre_off, n_roms, "ROM mappings");
    const uint32_t instr_off = (3 * n_roms + 1) & ~1u;   // 8-byte aligned counters
    c->stepw_words = instr_off + 9;
    c->instr_off = instr_off;
    for (auto& P : c->pipes) {
        if (!rc) rc = alloc_n(c, &P.d_stepw, c->stepw_words, "per-call counters");
        if (rc) break;
        P.d_counts = P.d_stepw;
        P.d_instr = reinterpret_cast<unsigned long long*>(P.d_stepw + instr_off);   // 4 counters
        P.d_queue = P.d_stepw + instr_off + 8;
    }
    if (!rc) rc = ensure_tile_buffer(c);
    if (rc) return rc;
    for (auto& P : c->pipes) HIP_OK(hipMemset(P.d_stepw, 0, (size_t)c->stepw_words * 4));
    HIP_OK(hipMemset(c->d_roms, 0, (size_t)n_roms * kRomSlot + 16));
    HIP_OK(hipMemcpy(c->d_roms, c->h_roms.data(), c->h_roms.size(), hipMemcpyHostToDevice));
    std::vector<CartMap> cmap(n_roms);
    std::vector<uint32_t> pre_off(n_roms);
    for (uint32_t r = 0; r < n_roms; ++r) {
        cmap[r] = pack_cart(c->h_rinfo[r]);
        pre_off[r] = c->h_rinfo[r].pre_off;
    }
    HIP_OK(hipMemcpy(c->d_cmap, cmap.data(), n_roms * sizeof(CartMap), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(c->d_pre_off, pre_off.data(), n_roms * 4, hipMemcpyHostToDevice));
    for (uint32_t r = 0; r < n_roms; ++r)
        launch_predecode(c->d_roms + (size_t)r * kRomSlot, c->h_rinfo[r], c->d_pre + c->h_rinfo[r].pre_off,
                         c->cfg.collisions ? 1u : 0u, nullptr);
    HIP_OK(hipGetLastError());
    HIP_OK(hipDeviceSynchronize());
    return VCS_OK;
}

// No-ops after the copy at assign time: every env runs the frame counts
// k_reset left in d_nf, in launches of at most max_batch envs (ROM-homogeneous
// tiles of 64 built on the host; output position = env - first env).
static int assign_noops(vcs_ctx* c, const uint16_t* d_nf, const uint16_t* env_rom_host) {
    const uint32_t N = c->cfg.num_envs, R = c->n_roms, C = c->max_batch;
    Tile* d_t = nullptr;
    StepInfo* d_info = nullptr;
    uint32_t* d_cnt = nullptr;
    const uint32_t cap = (C + kLanes - 1) / kLanes + R;
    int rc = alloc_n(c, &d_t, cap, "assign no-op tiles");
    if (!rc) rc = alloc_n(c, &d_info, C, "assign no-op info");
    if (!rc) rc = alloc_n(c, &d_cnt, 1, "assign no-op tile count");
    for (uint32_t c0 = 0; c0 < N && !rc; c0 += C) {
        const uint32_t cn = std::min(C, N - c0);
        std::vector<Tile> tl;
        for (uint32_t r = 0; r < R; ++r) {
            Tile t;
            std::memset(&t, 0xFF, sizeof(t));
            t.rom = (int32_t)r;
            t.count = 0;
            for (uint32_t e = c0; e < c0 + cn; ++e) {
                if (env_rom_host[e] != r) continue;
                t.env[t.count] = (int32_t)e;
                t.out[t.count] = (int32_t)(e - c0);
                if (++t.count == kLanes) {
                    tl.push_back(t);
                    std::memset(&t, 0xFF, sizeof(t));
                    t.rom = (int32_t)r;
                    t.count = 0;
                }
            }
            if (t.count) tl.push_back(t);
        }
        const uint32_t nt = (uint32_t)tl.size();
        if (hipMemcpy(d_t, tl.data(), (size_t)nt * sizeof(Tile), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(d_cnt, &nt, 4, hipMemcpyHostToDevice) != hipSuccess) {
            rc = fail(VCS_E_HIP, "assign no-op upload failed");
            break;
        }
        InterpArgs ia{};
        ia.tiles = d_t;
        ia.n_tiles = d_cnt;
        ia.envs = c->d_envs;
        ia.roms = c->d_roms;
        ia.cmap = c->d_cmap;
        ia.pre_off = c->d_pre_off;
        ia.pre = c->d_pre;
        ia.actions = nullptr;
        ia.nframes_per_out = d_nf + c0;
        ia.nframes = 0;
        ia.render_all = 0;
        ia.log_enabled = 0;
        ia.early_stop = 0;
        ia.sticky_thr = 0;
        ia.frameskip = c->cfg.frameskip;
        ia.seed = c->cfg.seed;
        ia.logs = nullptr;
        ia.n_slots = 2;
        ia.info = d_info;
        ia.reward = nullptr;
        ia.done = nullptr;
        ia.err_word = c->d_err;
        ia.instr_total = nullptr;
        ia.queue = nullptr;
        ia.track = c->cfg.collisions ? 1 : 0;
        ia.cx_logs = c->pipes[0].d_cxlogs;
        ia.count_step = 0;
        launch_interp(ia, nt, kLanes, c->rom_lds, nullptr);
        if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
            rc = fail(VCS_E_HIP, "assign no-op frames failed");
            break;
        }
    }
    dev_free(c, d_t, (size_t)cap * sizeof(Tile));
    dev_free(c, d_info, (size_t)C * sizeof(StepInfo));
    dev_free(c, d_cnt, 4);
    return rc;
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

    int rc = build_all_tiles(c);
    if (rc) return rc;
    ++c->generation;

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
            // no-ops after the copy: the entry stops two frames before the start-up's end
            nfr[r * K + k] = (uint16_t)(c->cfg.noop_after_copy ? c->cfg.startup_frames - 1
                                                               : 1 + c->cfg.startup_frames + noops);
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
    if (!rc) rc = alloc_n(c, &d_clog, (size_t)M * (2 + (c->cfg.collisions ? 1 : 0)) * kFrameLogBytes,
                          "cache row logs");
    if (!rc) rc = alloc_n(c, &d_cinfo, M, "cache info");
    if (!rc) rc = alloc_n(c, &d_cnt, 1, "cache tile count");
    auto cleanup = [&]() {
        dev_free(c, d_ct, ctiles.size() * sizeof(Tile));
        dev_free(c, d_nfr, (size_t)M * 2);
        dev_free(c, d_clog, (size_t)M * (2 + (c->cfg.collisions ? 1 : 0)) * kFrameLogBytes);
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
    ia.cmap = c->d_cmap;
    ia.pre_off = c->d_pre_off;
    ia.pre = c->d_pre;
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
    ia.track = c->cfg.collisions ? 1 : 0;
    ia.cx_logs = d_clog + (size_t)M * 2 * kFrameLogBytes;
    ia.count_step = 1;
    launch_interp(ia, n_ct, kLanes, c->rom_lds, nullptr);
    RenderArgs ra{};
    ra.logs = d_clog;
    ra.n_slots = 2;
    ra.info = d_cinfo;
    ra.frames = nullptr;
    ra.obs = c->d_cache_obs;
    ra.gray = c->d_gray;
    ra.n = M;
    ra.force_obs = 1;
    launch_render_obs(ra, 256, nullptr);
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
    uint16_t* d_nf = nullptr;
    if (c->cfg.noop_after_copy) {
        rc = alloc_n(c, &d_nf, N, "assign no-op frame counts");
        if (rc) return rc;
        rs.nfpo = d_nf;
        rs.noop_max = c->cfg.noop_max;
    }
    launch_reset(rs, nullptr);
    HIP_OK(hipGetLastError());
    if (c->cfg.noop_after_copy) {
        // each env runs its no-op frames, max_batch envs per launch (the
        // collision scratch is sized for that); no observation is kept
        rc = assign_noops(c, d_nf, env_rom_host);
        dev_free(c, d_nf, (size_t)N * 2);
        if (rc) return rc;
    }
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
    Pipe& P = c->pipes[0];
    ResetArgs rs{};
    rs.envs = c->d_envs;
    rs.ids = ids;
    rs.n = n;
    rs.num_envs = c->cfg.num_envs;
    rs.info = nullptr;
    rs.valid = nullptr;
    const Tile* tiles = c->d_tiles_all;
    const uint32_t* n_tiles = c->d_n_tiles_all;
    uint32_t grid = c->n_tiles_all;
    if (c->cfg.noop_after_copy && (ids || n != c->cfg.num_envs)) {
        // the no-op frames need tiles of the listed envs (validation included)
        launch_step_begin(P.d_stepw, c->stepw_words, P.d_tag, P.residue, s);
        int rc = build_tiles(c, P, ids, n, nullptr, nullptr, s, &grid);
        if (rc) return rc;
        tiles = P.d_tiles;
        n_tiles = P.d_n_tiles;
        rs.valid = P.d_valid;
    } else if (c->cfg.noop_after_copy) {
        launch_step_begin(P.d_stepw + c->instr_off, c->stepw_words - c->instr_off, nullptr, 0, s);
    } else if (ids) {
        launch_step_begin(P.d_counts, c->n_roms, P.d_tag, P.residue, s);
        launch_validate(ids, n, c->cfg.num_envs, c->d_env_rom, c->d_claim, P.d_tag, P.d_counts, P.d_valid,
                        nullptr, nullptr, nullptr, c->d_err, s);
        rs.valid = P.d_valid;
    }
    rs.cache_state = c->d_cache_state;
    rs.cache_obs = c->d_cache_obs;
    rs.K = c->cfg.reset_cache_k;
    rs.seed = c->cfg.seed;
    rs.obs = obs;
    rs.nfpo = c->cfg.noop_after_copy ? P.d_nfpo : nullptr;
    rs.noop_max = c->cfg.noop_max;
    begin_timed(c, 3, s);
    launch_reset(rs, s);
    end_timed(c, s);
    HIP_OK(hipGetLastError());
    if (c->cfg.noop_after_copy) return enqueue_noops(c, P, tiles, n_tiles, grid, n, obs, s);
    return VCS_OK;
}

int vcs_step(vcs_ctx* c, const int32_t* ids, const uint8_t* actions, uint32_t n, uint8_t* obs, int32_t* reward,
             uint8_t* done, uint8_t* frames, void* stream) {
    int rc = check_step_args(c, n, actions, reward, done);
    if (rc || n == 0) return rc;
    return enqueue_step(c, 0, ids, actions, n, obs, reward, done, frames, (hipStream_t)stream);
}

int vcs_step_pipe(vcs_ctx* c, uint32_t pipe, const int32_t* ids, const uint8_t* actions, uint32_t n, uint8_t* obs,
                  int32_t* reward, uint8_t* done, uint8_t* frames, void* stream) {
    int rc = check_step_args(c, n, actions, reward, done);
    if (rc || n == 0) return rc;
    if (pipe >= c->pipes.size()) return fail(VCS_E_INVAL, "no such pipeline");
    return enqueue_step(c, pipe, ids, actions, n, obs, reward, done, frames, (hipStream_t)stream);
}

int vcs_step_noalloc(vcs_ctx* c, const int32_t* ids, const uint8_t* actions, uint32_t n, uint8_t* obs,
                     int32_t* reward, uint8_t* done, void* stream) {
    if (!c) return fail(VCS_E_INVAL, "null context");
    if (!c->assigned) return fail(VCS_E_STATE, "vcs_assign first");
    if (n == 0) return VCS_OK;
    if (!actions || !reward || !done) return fail(VCS_E_INVAL, "actions, reward and done are required");
    if (n > kNoAllocEnvs) return fail(VCS_E_INVAL, "vcs_step_noalloc takes at most 512 envs per call");
    if (n > c->cfg.num_envs) return fail(VCS_E_INVAL, "n exceeds num_envs");
    if (c->cfg.noop_after_copy) return fail(VCS_E_INVAL, "vcs_step_noalloc does not run reset no-ops after the copy");
    if (c->n_roms > kNoAllocRoms) return fail(VCS_E_INVAL, "vcs_step_noalloc takes at most 1024 ROMs");
    if ((n + c->launch.tile_envs - 1) / c->launch.tile_envs + c->n_roms > kNoAllocTiles ||
        c->stepw_words > kNoAllocStepw)
        return fail(VCS_E_INVAL, "the call's tiles or counters exceed the static scratch");
    const int dev = c->cfg.device;
    if (dev < 0 || dev >= kMaxDevices || !g_scratch[dev]) return fail(VCS_E_STATE, "scratch address not taken");
    uint8_t* base = g_scratch[dev];   // the device address, never the array's host name
    Pipe P;
    P.d_logs = base + kScLogs;
    P.d_cxlogs = c->cfg.collisions ? base + kScCxLogs : nullptr;
    P.d_info = reinterpret_cast<StepInfo*>(base + kScInfo);
    P.d_valid = base + kScValid;
    P.d_tiles = reinterpret_cast<Tile*>(base + kScTiles);
    P.d_n_tiles = reinterpret_cast<uint32_t*>(base + kScNTiles);
    P.d_tag = reinterpret_cast<uint32_t*>(base + kScTag);
    P.residue = kScratchResidue;
    P.d_stepw = reinterpret_cast<uint32_t*>(base + kScStepw);
    P.d_counts = P.d_stepw;
    P.d_instr = reinterpret_cast<unsigned long long*>(P.d_stepw + c->instr_off);
    P.d_queue = P.d_stepw + c->instr_off + 8;
    // the step's kernels, with its counters and tiles cleared or rebuilt by
    // kernels; no event or buffer is created here
    const bool timing = c->timing;
    c->timing = false;
    hipStream_t s = (hipStream_t)stream;
    int rc = enqueue_sim_on(c, P, 2, false, ids, actions, n, obs, reward, done, nullptr, s);
    if (!rc) rc = enqueue_render_on(c, P, 2, n, obs, nullptr, s);
    c->timing = timing;
    return rc;
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
    const uint32_t bank = e.bank | ((uint32_t)e.bank_hi << 8);
    if (bank >= c->h_rinfo[e.rom_id].n_vbanks) return fail(VCS_E_INVAL, "bank state out of range for the ROM's scheme");
    e.track_cx = c->cfg.collisions ? 1 : 0;      // the context decides whether latches are tracked
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
    if (c->pipes[0].d_instr) HIP_OK(hipMemcpy(&v, c->pipes[0].d_instr, 8, hipMemcpyDeviceToHost));
    *out = v;
    return VCS_OK;
}

int vcs_last_step_stats(vcs_ctx* c, uint64_t* out2) {
    if (!c || !out2) return fail(VCS_E_INVAL, "null argument");
    HIP_OK(hipSetDevice(c->cfg.device));
    HIP_OK(hipDeviceSynchronize());
    unsigned long long v[2] = {0, 0};
    if (c->pipes[0].d_instr) HIP_OK(hipMemcpy(v, c->pipes[0].d_instr, 16, hipMemcpyDeviceToHost));
    out2[0] = v[0];
    out2[1] = v[1];
    return VCS_OK;
}

int vcs_last_step_counts(vcs_ctx* c, uint64_t* out4) {
    if (!c || !out4) return fail(VCS_E_INVAL, "null argument");
    HIP_OK(hipSetDevice(c->cfg.device));
    HIP_OK(hipDeviceSynchronize());
    unsigned long long v[4] = {0, 0, 0, 0};
    if (c->pipes[0].d_instr) HIP_OK(hipMemcpy(v, c->pipes[0].d_instr, 32, hipMemcpyDeviceToHost));
    for (int i = 0; i < 4; ++i) out4[i] = v[i];
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

int vcs_set_launch(vcs_ctx* c, const vcs_launch* l) {
    if (!c || !l) return fail(VCS_E_INVAL, "null argument");
    int rc = check_launch(l);
    if (rc) return rc;
    HIP_OK(hipSetDevice(c->cfg.device));
    HIP_OK(hipDeviceSynchronize());
    const vcs_launch old = c->launch;
    c->launch = *l;
    if (c->n_roms) {
        rc = ensure_tile_buffer(c);
        if (!rc && c->assigned && l->tile_envs != old.tile_envs) rc = build_all_tiles(c);
        if (rc) {
            c->launch = old;
            return rc;
        }
    }
    ++c->generation;
    return VCS_OK;
}

int vcs_get_launch(vcs_ctx* c, vcs_launch* out) {
    if (!c || !out) return fail(VCS_E_INVAL, "null argument");
    *out = c->launch;
    return VCS_OK;
}

int vcs_autotune(vcs_ctx* c, uint32_t n, uint32_t steps, int want_frames, int want_obs, vcs_launch* best_out,
                 double* best_ms_out) {
    if (!c) return fail(VCS_E_INVAL, "null context");
    if (!c->assigned) return fail(VCS_E_STATE, "vcs_assign first");
    if (n == 0) n = c->max_batch;
    if (n > c->max_batch) return fail(VCS_E_INVAL, "n exceeds max_batch");
    if (steps == 0 || steps > 1000) return fail(VCS_E_INVAL, "steps must be in [1, 1000]");
    HIP_OK(hipSetDevice(c->cfg.device));
    HIP_OK(hipDeviceSynchronize());
    const uint32_t N = c->cfg.num_envs;
    const vcs_launch start = c->launch;

    // temporaries: env-state snapshot, outputs, actions
    DevEnv* d_backup = nullptr;
    uint8_t *d_obs = nullptr, *d_done = nullptr, *d_frames = nullptr, *d_act = nullptr;
    int32_t* d_rew = nullptr;
    const size_t frame_bytes = (size_t)n * c->n_slots * kFrameBytes;
    int rc = alloc_n(c, &d_backup, N, "autotune state snapshot");
    if (!rc) rc = alloc_n(c, &d_rew, n, "autotune reward");
    if (!rc) rc = alloc_n(c, &d_done, n, "autotune done");
    if (!rc) rc = alloc_n(c, &d_act, (size_t)(steps + 1) * n, "autotune actions");
    if (!rc && want_obs) rc = alloc_n(c, &d_obs, (size_t)n * kObsBytes, "autotune obs");
    if (!rc && want_frames) rc = alloc_n(c, &d_frames, frame_bytes, "autotune frames");
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    uint32_t err_host[2] = {0, 0xFFFFFFFFu};
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
        dev_free(c, d_backup, (size_t)N * sizeof(DevEnv));
        dev_free(c, d_rew, (size_t)n * 4);
        dev_free(c, d_done, n);
        dev_free(c, d_act, (size_t)(steps + 1) * n);
        dev_free(c, d_obs, (size_t)n * kObsBytes);
        dev_free(c, d_frames, frame_bytes);
    };
    if (rc) {
        cleanup();
        return rc;
    }
    {
        std::vector<uint8_t> act((size_t)(steps + 1) * n);
        uint64_t z = c->cfg.seed ^ 0x5EED5EEDull;
        for (auto& a : act) a = (uint8_t)((mix64(z += kGamma) >> 32) % VCS_N_ACTIONS);
        if (hipMemcpy(d_act, act.data(), act.size(), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(d_backup, c->d_envs, (size_t)N * sizeof(DevEnv), hipMemcpyDeviceToDevice) != hipSuccess ||
            hipMemcpy(err_host, c->d_err, 8, hipMemcpyDeviceToHost) != hipSuccess ||
            hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
            hipEventCreate(&e1) != hipSuccess) {
            cleanup();
            return fail(VCS_E_HIP, "autotune set-up failed");
        }
    }
    const bool timing = c->timing;
    c->timing = false;
    // time one candidate: same start states, 1 untimed step then `steps` timed steps
    auto measure = [&](const vcs_launch& l, double* ms) -> int {
        c->launch = l;
        int r = ensure_tile_buffer(c);
        if (!r) r = build_all_tiles(c);
        if (r) return r;
        HIP_OK(hipMemcpyAsync(c->d_envs, d_backup, (size_t)N * sizeof(DevEnv), hipMemcpyDeviceToDevice, s));
        for (uint32_t k = 0; k <= steps; ++k) {
            if (k == 1) HIP_OK(hipEventRecord(e0, s));
            r = enqueue_step(c, 0, nullptr, d_act + (size_t)k * n, n, d_obs, d_rew, d_done, d_frames, s);
            if (r) return r;
        }
        HIP_OK(hipEventRecord(e1, s));
        HIP_OK(hipEventSynchronize(e1));
        float t = 0;
        HIP_OK(hipEventElapsedTime(&t, e0, e1));
        *ms = t / steps;
        return VCS_OK;
    };
    vcs_launch best = start;
    best.workers = 0;
    double best_ms = 1e30;
    // interpreter shapes: a later candidate must be 3 % faster (near ties keep
    // the wider, fewer-workgroup shape); render blocks: the fastest
    auto consider = [&](const vcs_launch& l, double margin) -> int {
        double ms = 0;
        int r = measure(l, &ms);
        if (r == VCS_E_BUDGET) return VCS_OK;   // this shape's tile tables do not fit: skip it
        if (r) return r;
        if (ms < best_ms * (1.0 - margin)) {
            best_ms = ms;
            best = l;
        }
        return VCS_OK;
    };
    // 1) envs per wave (one workgroup per tile): widths whose tiles fit on the
    //    chip at once (up to 12 waves per CU with tiles of 32 envs or fewer)
    for (uint32_t w = 64; w >= 1 && !rc; w >>= 1) {
        const uint64_t tiles = (n + w - 1) / w + c->n_roms;
        if (w != 64 && tiles > 12ull * c->n_cu) break;
        vcs_launch l{w, 0, start.render_block};
        rc = consider(l, 0.03);
    }
    // 2) persistent interpreter with 1, 2, 4 or 8 workgroups per CU
    const uint64_t tiles_best = (n + best.tile_envs - 1) / best.tile_envs + c->n_roms;
    for (uint32_t k = 1; k <= 8 && !rc; k <<= 1) {
        if ((uint64_t)k * c->n_cu >= tiles_best) break;
        vcs_launch l = best;
        l.workers = k * c->n_cu;
        rc = consider(l, 0.03);
    }
    // 3) render workgroup size
    if (!rc && (want_frames || want_obs)) {
        const vcs_launch b = best;
        for (uint32_t blk : {128u, 256u, 512u}) {
            if (blk == b.render_block || rc) continue;
            vcs_launch l = b;
            l.render_block = blk;
            rc = consider(l, 0.0);
        }
    }
    c->timing = timing;
    // restore the env states and error word whatever happened, keep the best shape
    hipError_t he = hipStreamSynchronize(s);
    if (he == hipSuccess) he = hipMemcpy(c->d_envs, d_backup, (size_t)N * sizeof(DevEnv), hipMemcpyDeviceToDevice);
    if (he == hipSuccess) he = hipMemcpy(c->d_err, err_host, 8, hipMemcpyHostToDevice);
    for (auto& P : c->pipes)
        if (he == hipSuccess) he = hipMemset(P.d_stepw, 0, (size_t)c->stepw_words * 4);
    c->launch = rc ? start : best;
    int rc2 = ensure_tile_buffer(c);
    if (!rc2) rc2 = build_all_tiles(c);
    ++c->generation;
    cleanup();
    if (rc) return rc;
    if (he != hipSuccess) return fail(VCS_E_HIP, std::string("autotune restore failed: ") + hipGetErrorString(he));
    if (rc2) return rc2;
    if (best_out) *best_out = best;
    if (best_ms_out) *best_ms_out = best_ms;
    return VCS_OK;
}

struct vcs_graph {
    vcs_ctx* c = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t generation = 0;
};

int vcs_graph_create(vcs_ctx* c, const int32_t* ids, const uint8_t* actions, uint32_t n, uint32_t steps,
                     uint8_t* obs, int32_t* reward, uint8_t* done, uint8_t* frames, vcs_graph** out) {
    if (!out) return fail(VCS_E_INVAL, "null argument");
    *out = nullptr;
    int rc = check_step_args(c, n, actions, reward, done);
    if (rc) return rc;
    if (n == 0) return fail(VCS_E_INVAL, "a graph needs n >= 1");
    if (steps == 0 || steps > 64) return fail(VCS_E_INVAL, "steps must be in [1, 64]");
    HIP_OK(hipSetDevice(c->cfg.device));
    hipStream_t s = nullptr;
    HIP_OK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    hipError_t he = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (he != hipSuccess) {
        (void)hipStreamDestroy(s);
        return fail(VCS_E_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(he));
    }
    const bool timing = c->timing;
    c->timing = false;
    // With two or more pipelines, step j runs on pipeline j % 2 and its render
    // goes on a second stream: it overlaps step j+1's interpreter, and step
    // j+2 (same pipeline scratch) waits for it.
    const bool overlap = c->pipes.size() >= 2 && steps >= 2;
    hipStream_t r = nullptr;
    std::vector<hipEvent_t> ev;
    auto evt = [&]() -> hipEvent_t {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        ev.push_back(e);
        return e;
    };
    if (overlap && hipStreamCreateWithFlags(&r, hipStreamNonBlocking) != hipSuccess) rc = fail(VCS_E_HIP, "stream");
    std::vector<hipEvent_t> rendered(steps, nullptr);
    for (uint32_t j = 0; j < steps && !rc; ++j) {
        uint8_t* ob = obs ? obs + (size_t)j * n * kObsBytes : nullptr;
        uint8_t* fr = frames ? frames + (size_t)j * n * c->n_slots * kFrameBytes : nullptr;
        if (!overlap) {
            rc = enqueue_step(c, 0, ids, actions + (size_t)j * n, n, ob, reward + (size_t)j * n, done + (size_t)j * n,
                              fr, s);
            continue;
        }
        const uint32_t p = j % 2;
        if (j >= 2 && hipStreamWaitEvent(s, rendered[j - 2], 0) != hipSuccess) rc = fail(VCS_E_HIP, "wait");
        if (!rc) rc = enqueue_sim(c, p, ids, actions + (size_t)j * n, n, ob, reward + (size_t)j * n, done + (size_t)j * n,
                                  fr, s);
        hipEvent_t simd = rc ? nullptr : evt();
        if (!rc && (!simd || hipEventRecord(simd, s) != hipSuccess || hipStreamWaitEvent(r, simd, 0) != hipSuccess))
            rc = fail(VCS_E_HIP, "event");
        if (!rc) rc = enqueue_render(c, p, n, ob, fr, r);
        if (!rc) {
            rendered[j] = evt();
            if (!rendered[j] || hipEventRecord(rendered[j], r) != hipSuccess) rc = fail(VCS_E_HIP, "event");
        }
    }
    if (overlap && !rc) {   // join the render stream back into the captured stream
        for (uint32_t j = steps - 2; j < steps && !rc; ++j)
            if (hipStreamWaitEvent(s, rendered[j], 0) != hipSuccess) rc = fail(VCS_E_HIP, "join");
    }
    c->timing = timing;
    hipGraph_t g = nullptr;
    he = hipStreamEndCapture(s, &g);
    (void)hipStreamDestroy(s);
    if (r) (void)hipStreamDestroy(r);
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    if (rc || he != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : fail(VCS_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(he));
    }
    hipGraphExec_t x = nullptr;
    he = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (he != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(VCS_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(he));
    }
    vcs_graph* G = new vcs_graph();
    G->c = c;
    G->graph = g;
    G->exec = x;
    G->generation = c->generation;
    *out = G;
    return VCS_OK;
}

int vcs_graph_launch(vcs_graph* g, void* stream) {
    if (!g) return fail(VCS_E_INVAL, "null graph");
    if (g->generation != g->c->generation)
        return fail(VCS_E_STATE, "the context's ROMs, envs or launch shape changed since the graph was captured");
    HIP_OK(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return VCS_OK;
}

void vcs_graph_destroy(vcs_graph* g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

struct vcs_stack {
    vcs_ctx* c = nullptr;
    uint8_t* ring = nullptr;
    uint8_t* head = nullptr;
    uint32_t depth = 0, bits = 0;
    size_t ring_bytes = 0;
};

int vcs_stack_create(vcs_ctx* c, uint32_t depth, uint32_t bits, vcs_stack** out) {
    if (!c || !out) return fail(VCS_E_INVAL, "null argument");
    *out = nullptr;
    if (depth < 1 || depth > 16) return fail(VCS_E_INVAL, "depth must be in [1, 16]");
    if (bits != 8 && bits != 4) return fail(VCS_E_INVAL, "bits must be 8 or 4");
    HIP_OK(hipSetDevice(c->cfg.device));
    vcs_stack* S = new vcs_stack();
    S->c = c;
    S->depth = depth;
    S->bits = bits;
    S->ring_bytes = (size_t)c->cfg.num_envs * depth * (bits == 4 ? kObsBytes / 2 : kObsBytes);
    int rc = alloc_n(c, &S->ring, S->ring_bytes, "frame stack");
    if (!rc) rc = alloc_n(c, &S->head, c->cfg.num_envs, "frame stack heads");
    if (!rc && (hipMemset(S->ring, 0, S->ring_bytes) != hipSuccess ||
                hipMemset(S->head, 0, c->cfg.num_envs) != hipSuccess || hipDeviceSynchronize() != hipSuccess))
        rc = fail(VCS_E_HIP, "frame stack clear failed");
    if (rc) {
        vcs_stack_destroy(S);
        return rc;
    }
    *out = S;
    return VCS_OK;
}

int vcs_stack_push(vcs_stack* S, const int32_t* ids, uint32_t n, const uint8_t* obs, const uint8_t* done,
                   uint8_t* out, void* stream) {
    if (!S) return fail(VCS_E_INVAL, "null stack");
    if (n > S->c->cfg.num_envs) return fail(VCS_E_INVAL, "n exceeds num_envs");
    if (n == 0) return VCS_OK;
    if (!obs) return fail(VCS_E_INVAL, "obs is required");
    launch_stack(S->ring, S->head, ids, n, S->c->cfg.num_envs, S->depth, S->bits, obs, done, out,
                 (hipStream_t)stream);
    HIP_OK(hipGetLastError());
    return VCS_OK;
}

void vcs_stack_destroy(vcs_stack* S) {
    if (!S) return;
    (void)hipSetDevice(S->c->cfg.device);
    (void)hipDeviceSynchronize();
    dev_free(S->c, S->ring, S->ring_bytes);
    dev_free(S->c, S->head, S->c->cfg.num_envs);
    delete S;
}

namespace {
// the policy network's layers: input side, kernel, stride, channels
struct LayerShape {
    uint32_t H, Cin, KW, stride, OH, N, Npad;
};
constexpr LayerShape kLayers[5] = {
    {84, 4, 8, 4, 20, 32, 32},     // conv 32 x 8x8 / 4 on the u8 stack
    {20, 32, 4, 2, 9, 64, 64},     // conv 64 x 4x4 / 2
    {9, 64, 3, 1, 7, 64, 64},      // conv 64 x 3x3 / 1
    {7, 64, 7, 1, 1, 512, 512},    // 3136 -> 512 as a 7x7 convolution
    {1, 512, 1, 1, 1, 19, 32},     // 512 -> 18 logits + value
};
constexpr uint32_t layer_k(const LayerShape& L) { return L.KW * L.KW * L.Cin; }
}  // namespace

struct vcs_policy {
    vcs_ctx* c = nullptr;
    uint16_t* w[5] = {};
    float* b[5] = {};
    uint16_t* act[4] = {};   // outputs of layers 1-4
    float* logits = nullptr;
    uint32_t max_n = 0;
    std::vector<std::pair<void*, size_t>> allocs;
};

int vcs_policy_create(vcs_ctx* c, const uint16_t* const* w_host, const float* const* b_host, vcs_policy** out) {
    if (!c || !w_host || !b_host || !out) return fail(VCS_E_INVAL, "null argument");
    *out = nullptr;
    for (int l = 0; l < 5; ++l)
        if (!w_host[l] || !b_host[l]) return fail(VCS_E_INVAL, "null weight or bias array");
    HIP_OK(hipSetDevice(c->cfg.device));
    vcs_policy* P = new vcs_policy();
    P->c = c;
    P->max_n = c->max_batch;
    int rc = VCS_OK;
    auto take = [&](void** p, size_t bytes, const char* what) {
        if (!rc) rc = dev_alloc(c, p, bytes, what);
        if (!rc) P->allocs.push_back({*p, bytes});
    };
    for (int l = 0; l < 5 && !rc; ++l) {
        const LayerShape& L = kLayers[l];
        const size_t K = layer_k(L);
        take(reinterpret_cast<void**>(&P->w[l]), (size_t)L.Npad * K * 2, "policy weights");
        take(reinterpret_cast<void**>(&P->b[l]), (size_t)L.Npad * 4, "policy biases");
        if (rc) break;
        // rows past N are zero; the device copy is in operand order
        std::vector<uint16_t> wz((size_t)L.Npad * K, 0);
        std::vector<float> bz(L.Npad, 0.f);
        for (uint32_t cch = 0; cch < L.N; ++cch)
            for (size_t k = 0; k < K; ++k)
                wz[policy_swizzle_index(cch, (uint32_t)k, L.Npad / 16)] = w_host[l][(size_t)cch * K + k];
        std::memcpy(bz.data(), b_host[l], (size_t)L.N * 4);
        if (hipMemcpy(P->w[l], wz.data(), wz.size() * 2, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(P->b[l], bz.data(), bz.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
            rc = fail(VCS_E_HIP, "policy weight upload failed");
    }
    for (int l = 0; l < 4 && !rc; ++l) {
        const LayerShape& L = kLayers[l];
        take(reinterpret_cast<void**>(&P->act[l]), (size_t)P->max_n * L.OH * L.OH * L.N * 2, "policy activations");
    }
    take(reinterpret_cast<void**>(&P->logits), (size_t)P->max_n * 32 * 4, "policy logits");
    if (rc) {
        vcs_policy_destroy(P);
        return rc;
    }
    *out = P;
    return VCS_OK;
}

int vcs_policy_act(vcs_policy* P, const uint8_t* stack, uint32_t n, float* logits, uint8_t* actions, void* stream) {
    if (!P) return fail(VCS_E_INVAL, "null policy");
    if (n > P->max_n) return fail(VCS_E_INVAL, "n exceeds max_batch");
    if (n == 0) return VCS_OK;
    if (!stack || (!logits && !actions)) return fail(VCS_E_INVAL, "stack and an output are required");
    hipStream_t s = (hipStream_t)stream;
    float* lg = logits ? logits : P->logits;
    const void* in = stack;
    for (int l = 0; l < 5; ++l) {
        const LayerShape& L = kLayers[l];
        PolicyLayerArgs a{};
        a.in = in;
        a.w = P->w[l];
        a.bias = P->b[l];
        a.out = l < 4 ? static_cast<void*>(P->act[l]) : static_cast<void*>(lg);
        a.M = n * L.OH * L.OH;
        launch_policy_layer(l, a, s);
        in = a.out;
    }
    if (actions) launch_argmax(lg, n, actions, s);
    HIP_OK(hipGetLastError());
    return VCS_OK;
}

void vcs_policy_destroy(vcs_policy* P) {
    if (!P) return;
    (void)hipSetDevice(P->c->cfg.device);
    (void)hipDeviceSynchronize();
    for (auto& a : P->allocs) dev_free(P->c, a.first, a.second);
    delete P;
}

}  // extern "C"
