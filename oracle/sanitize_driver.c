/*
 * Standalone driver of the CPU oracle -- TEST INFRASTRUCTURE.
 *
 * Built by the test suite with gcc under AddressSanitizer and
 * UndefinedBehaviorSanitizer (host code only; the oracle has no GPU code),
 * it runs one env workload read from a binary job file through the oracle's
 * C API and prints a digest of everything the workload produced, so the test
 * can compare the instrumented build with the ordinary shared library.
 *
 * Job file (little-endian):
 *   u32 n_roms; per ROM: u32 scheme, u32 bytes, bytes of ROM
 *   u32 num_envs, frameskip, sticky_threshold, render_mode, collisions,
 *       noop_after_copy, steps; u64 seed
 *   u8 gray_lut[128]; u16 env_rom[num_envs]; u8 actions[steps][num_envs]
 * Output (stdout): one line per step "step s <reward sum> <done count>
 * <fnv1a of obs> <fnv1a of frames>", then one line per env "state e <fnv1a of
 * its state record>", then "errors <first env> <bits>".
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "vcs_oracle.h"

static uint64_t fnv1a(const uint8_t* p, size_t n, uint64_t h) {
    for (size_t i = 0; i < n; i++) {
        h ^= p[i];
        h *= 0x100000001B3ull;
    }
    return h;
}

static int rd(FILE* f, void* p, size_t n) { return fread(p, 1, n, f) == n ? 0 : -1; }

int main(int argc, char** argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s job-file\n", argv[0]);
        return 2;
    }
    FILE* f = fopen(argv[1], "rb");
    if (!f) {
        perror(argv[1]);
        return 2;
    }
    uint32_t n_roms = 0;
    if (rd(f, &n_roms, 4) || n_roms == 0 || n_roms > 64) return 3;
    uint8_t** roms = calloc(n_roms, sizeof(uint8_t*));
    uint32_t* sizes = calloc(n_roms, sizeof(uint32_t));
    uint32_t* schemes = calloc(n_roms, sizeof(uint32_t));
    for (uint32_t r = 0; r < n_roms; r++) {
        if (rd(f, &schemes[r], 4) || rd(f, &sizes[r], 4) || sizes[r] > (1u << 20)) return 3;
        roms[r] = malloc(sizes[r]);
        if (rd(f, roms[r], sizes[r])) return 3;
    }
    uint32_t hdr[7];
    uint64_t seed;
    oracle_config cfg;
    memset(&cfg, 0, sizeof cfg);
    if (rd(f, hdr, sizeof hdr) || rd(f, &seed, 8) || rd(f, cfg.gray_lut, 128)) return 3;
    cfg.num_envs = hdr[0];
    cfg.frameskip = hdr[1];
    cfg.sticky_threshold = hdr[2];
    cfg.render_mode = hdr[3];
    cfg.collisions = hdr[4];
    cfg.noop_after_copy = hdr[5];
    cfg.reset_cache_k = 30;
    cfg.noop_max = 30;
    cfg.startup_frames = 64;
    cfg.seed = seed;
    const uint32_t n = cfg.num_envs, steps = hdr[6];
    uint16_t* env_rom = malloc(sizeof(uint16_t) * n);
    uint8_t* actions = malloc((size_t)steps * n);
    if (rd(f, env_rom, sizeof(uint16_t) * n) || rd(f, actions, (size_t)steps * n)) return 3;
    fclose(f);

    oracle_ctx* ctx = NULL;
    if (oracle_create(&cfg, &ctx) != ORC_OK) return 4;
    if (oracle_load_roms(ctx, n_roms, (const uint8_t* const*)roms, sizes, schemes) != ORC_OK) return 5;
    if (oracle_assign(ctx, env_rom) != ORC_OK) return 6;
    const uint32_t slots = cfg.render_mode == ORC_RENDER_ALL ? cfg.frameskip : 2;
    const size_t fbytes = (size_t)n * slots * ORC_FRAME_H * ORC_FRAME_W;
    uint8_t* obs = malloc((size_t)n * ORC_OBS * ORC_OBS);
    uint8_t* frames = malloc(fbytes);
    int32_t* reward = malloc(sizeof(int32_t) * n);
    uint8_t* done = malloc(n);
    for (uint32_t s = 0; s < steps; s++) {
        if (oracle_step(ctx, NULL, actions + (size_t)s * n, n, obs, reward, done, frames, 1) != ORC_OK) return 7;
        long long rsum = 0;
        uint32_t dsum = 0;
        for (uint32_t e = 0; e < n; e++) {
            rsum += reward[e];
            dsum += done[e];
        }
        printf("step %u %lld %u %016llx %016llx\n", s, rsum, dsum,
               (unsigned long long)fnv1a(obs, (size_t)n * ORC_OBS * ORC_OBS, 0xCBF29CE484222325ull),
               (unsigned long long)fnv1a(frames, fbytes, 0xCBF29CE484222325ull));
    }
    uint8_t st[ORC_STATE_BYTES];
    for (uint32_t e = 0; e < n; e++) {
        if (oracle_get_state(ctx, e, st) != ORC_OK) return 8;
        printf("state %u %016llx\n", e, (unsigned long long)fnv1a(st, sizeof st, 0xCBF29CE484222325ull));
    }
    uint32_t first = 0, bits = 0;
    oracle_poll_errors(ctx, &first, &bits);
    printf("errors %u %u\n", first, bits);
    oracle_destroy(ctx);
    for (uint32_t r = 0; r < n_roms; r++) free(roms[r]);
    free(roms);
    free(sizes);
    free(schemes);
    free(env_rom);
    free(actions);
    free(obs);
    free(frames);
    free(reward);
    free(done);
    return 0;
}
