// TIA render and observation kernels.
//
// What they compute (paper, Section 3): the "TIA kernel" that turns the
// logged register writes into the 160x210 frame, run only for frames that are
// needed -- the observation is the pixelwise maximum of the last two frames
// of the step.  Unlike the paper's one-thread-per-game TIA kernel, rows are
// drawn in parallel (the paper names this as future work): each thread draws
// one row from the row's snapshot and the writes logged inside it, 16 pixels
// at a time, applying each write once.
//
// Pixel rule (TIA register semantics; the objects as in tia_draw.h): VBLANK
// D1, an early HMOVE's blank (pixels 0-7) or a pixel outside the frame -> 0;
// priority P0/M0 > P1/M1 > PF/BL > BK, or PF/BL > P0/M0 > P1/M1 > BK with
// CTRLPF D2; P0 and M0 in COLUP0, P1 and M1 in COLUP1, the ball in COLUPF,
// the playfield in COLUPF or, in score mode, COLUP0 / COLUP1 by half; the
// stored value is the colour & $FE.
//
// Observation: gray = lut[colour >> 1]; m = max over the two frames;
// obs[i][j] = floor((sum_r sum_c wr*wc*m[r][c] + 100) / 200), the exact-area
// average of 210x160 -> 84x84 with row weights in half rows (2,2,1 / 1,2,2)
// and column weights |[40j, 40j+40) & [21c, 21c+21)|, rounded half up.
#include "tia_draw.h"

namespace vcs {

// Segments are drawn 16 pixels at a time with bit masks: a 16-bit mask per
// object (bit i = pixel x0 + i), widened to byte masks and combined with one
// bitfield select per priority level.  A segment is split into runs at the
// in-row register writes that land inside it.

// four mask bits -> four byte masks (bit j -> 0xFF in byte j)
__device__ __forceinline__ uint32_t byte_masks(uint32_t n) { return ((n * 0x00204081u) & 0x01010101u) * 0xFFu; }

// (m & a) | (~m & b)
__device__ __forceinline__ uint32_t pick(uint32_t m, uint32_t a, uint32_t b) { return (m & a) | (~m & b); }

// What a drawn pixel holds, as a word of four equal bytes: the colour index
// (frames), or its gray level from the lookup table (observations: drawing
// gray directly takes one table read per colour register instead of one per
// pixel).
struct ColourPal {
    __device__ __forceinline__ uint32_t byte(uint32_t c) const { return c & 0xFE; }
    __device__ __forceinline__ uint32_t operator()(uint32_t c) const { return byte(c) * 0x01010101u; }
};
struct GrayPal {
    const uint8_t* lut;       // 128 entries in LDS
    __device__ __forceinline__ uint32_t byte(uint32_t c) const { return lut[(c & 0xFE) >> 1]; }
    __device__ __forceinline__ uint32_t operator()(uint32_t c) const { return byte(c) * 0x01010101u; }
};

// The common case's per-row state (what only a register write changes),
// computed when a row starts and again after its writes: whether the common
// case holds, the blank, the two sprites as drawn, and the colour of each
// combination of objects as a byte table, index P0 << 2 | P1 << 1 | PF, for
// the left and the right half (score mode colours the playfield by half).
struct PlainRow {
    uint32_t plain, blank;
    uint32_t s0, s1, p0x, p1x;
    uint32_t lo_l, hi_l, lo_r, hi_r;      // table bytes 0-3 / 4-7
};

template <class Pal>
__device__ __forceinline__ void plain_row(PlainRow& ps, const Regs& r, const Pal& pal) {
    ps.plain = (!(rb<R_FLAGS>(r) & 0x7F) && !((rb<R_NUSIZ0>(r) | rb<R_NUSIZ1>(r)) & 7) && rb<R_HMB>(r) == 0) ? 1u : 0u;
    ps.blank = (r.outside || (rb<R_VBLANK>(r) & 2)) ? 1u : 0u;
    const uint32_t g0 = rb<R_GRP0>(r), g1 = rb<R_GRP1>(r);
    ps.s0 = (rb<R_REFP0>(r) & 8) ? g0 : (__builtin_bitreverse32(g0) >> 24);
    ps.s1 = (rb<R_REFP1>(r) & 8) ? g1 : (__builtin_bitreverse32(g1) >> 24);
    ps.p0x = rb<R_P0X>(r);
    ps.p1x = rb<R_P1X>(r);
    const uint32_t ctrlpf = rb<R_CTRLPF>(r);
    const uint32_t c0 = pal.byte(rb<R_COLUP0>(r)), c1 = pal.byte(rb<R_COLUP1>(r));
    const uint32_t cf = pal.byte(rb<R_COLUPF>(r)), cb = pal.byte(rb<R_COLUBK>(r));
    const uint32_t cl = (ctrlpf & 2) ? c0 : cf, cr = (ctrlpf & 2) ? c1 : cf;
    if (ctrlpf & 4) {        // PF above the players: indices with PF set take the playfield colour
        ps.lo_l = cb | (cl << 8) | (c1 << 16) | (cl << 24);
        ps.hi_l = c0 | (cl << 8) | (c0 << 16) | (cl << 24);
        ps.lo_r = cb | (cr << 8) | (c1 << 16) | (cr << 24);
        ps.hi_r = c0 | (cr << 8) | (c0 << 16) | (cr << 24);
    } else {                 // P0 > P1 > PF > BK
        ps.lo_l = cb | (cl << 8) | (c1 << 16) | (c1 << 24);
        ps.lo_r = cb | (cr << 8) | (c1 << 16) | (c1 << 24);
        ps.hi_l = ps.hi_r = c0 * 0x01010101u;
    }
}

// bit j of the 4-bit n -> bit 0 of byte j
__device__ __forceinline__ uint32_t spread4(uint32_t n) { return (n * 0x00204081u) & 0x01010101u; }

// the 16 pixels x0 .. x0+15 of the common case from the per-row state: per
// 4 pixels, each byte's table index from the three masks, then one byte
// permute through the table
__device__ __forceinline__ uint4 draw16_row(const PlainRow& ps, const Regs& r, uint32_t x0) {
    if (ps.blank) return make_uint4(0, 0, 0, 0);
    const bool right = x0 >= 80;
    uint32_t n;
    if (!right) n = (r.pfm >> (x0 >> 2)) & 0xF;
    else if (!(rb<R_CTRLPF>(r) & 1)) n = (r.pfm >> ((x0 - 80) >> 2)) & 0xF;
    else n = rev4((r.pfm >> (16 - ((x0 - 80) >> 2))) & 0xF);
    const uint32_t m0 = window16s(ps.s0, 8, ps.p0x, x0), m1 = window16s(ps.s1, 8, ps.p1x, x0);
    const uint32_t lo = right ? ps.lo_r : ps.lo_l, hi = right ? ps.hi_r : ps.hi_l;
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        // a playfield bit covers one 4-pixel word: its index bit in all four bytes
        const uint32_t sel = (((n >> k) & 1) * 0x01010101u) | (spread4((m1 >> (4 * k)) & 0xF) << 1) |
                             (spread4((m0 >> (4 * k)) & 0xF) << 2);
        w[k] = __builtin_amdgcn_perm(hi, lo, sel);
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// the 16 pixels of the common case: one copy of each player at normal width,
// no missile, no ball, no vertical delay, no HMOVE blank
template <class Pal>
__device__ __forceinline__ uint4 draw16_plain(const Regs& r, uint32_t x0, const Pal& pal) {
    if (r.outside || (rb<R_VBLANK>(r) & 2)) return make_uint4(0, 0, 0, 0);
    const bool right = x0 >= 80;
    const uint32_t ctrlpf = rb<R_CTRLPF>(r);
    uint32_t n;
    if (!right) n = (r.pfm >> (x0 >> 2)) & 0xF;
    else if (!(ctrlpf & 1)) n = (r.pfm >> ((x0 - 80) >> 2)) & 0xF;
    else n = rev4((r.pfm >> (16 - ((x0 - 80) >> 2))) & 0xF);
    const uint32_t mpf = ((n & 1) | ((n & 2) << 3) | ((n & 4) << 6) | ((n & 8) << 9)) * 0xF;
    const uint32_t g0 = rb<R_GRP0>(r), g1 = rb<R_GRP1>(r);
    const uint32_t s0 = (rb<R_REFP0>(r) & 8) ? g0 : (__builtin_bitreverse32(g0) >> 24);
    const uint32_t s1 = (rb<R_REFP1>(r) & 8) ? g1 : (__builtin_bitreverse32(g1) >> 24);
    const uint32_t m0 = window16s(s0, 8, rb<R_P0X>(r), x0), m1 = window16s(s1, 8, rb<R_P1X>(r), x0);
    const uint32_t pfc = (ctrlpf & 2) ? (right ? rb<R_COLUP1>(r) : rb<R_COLUP0>(r)) : rb<R_COLUPF>(r);
    const uint32_t c0 = pal(rb<R_COLUP0>(r)), c1 = pal(rb<R_COLUP1>(r));
    const uint32_t cp = pal(pfc), cb = pal(rb<R_COLUBK>(r));
    const bool pf_first = (ctrlpf & 4) != 0;
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t b0 = byte_masks((m0 >> (4 * k)) & 0xF), b1 = byte_masks((m1 >> (4 * k)) & 0xF);
        const uint32_t bp = byte_masks((mpf >> (4 * k)) & 0xF);
        w[k] = pf_first ? pick(bp, cp, pick(b0, c0, pick(b1, c1, cb))) : pick(b0, c0, pick(b1, c1, pick(bp, cp, cb)));
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// the 16 pixels x0 .. x0+15 of row `row` drawn with registers r
template <class Pal>
__device__ __forceinline__ uint4 draw16(const Regs& r, uint32_t x0, uint32_t row, const Pal& pal) {
    // ENAM0/1, ENABL and its copy, the VDEL bits clear, both NUSIZ modes 0, no blank
    if (!(rb<R_FLAGS>(r) & 0x7F) && !((rb<R_NUSIZ0>(r) | rb<R_NUSIZ1>(r)) & 7) && rb<R_HMB>(r) == 0)
        return draw16_plain(r, x0, pal);
    uint32_t o[6], shown;
    objects16(r, x0, row, o, shown);
    if (!shown) return make_uint4(0, 0, 0, 0);
    const bool right = x0 >= 80;
    const uint32_t ctrlpf = rb<R_CTRLPF>(r);
    const uint32_t pfc = (ctrlpf & 2) ? (right ? rb<R_COLUP1>(r) : rb<R_COLUP0>(r)) : rb<R_COLUPF>(r);
    const uint32_t c0 = pal(rb<R_COLUP0>(r)), c1 = pal(rb<R_COLUP1>(r));
    const uint32_t cp = pal(pfc), cf = pal(rb<R_COLUPF>(r));
    const uint32_t cb = pal(rb<R_COLUBK>(r));
    const uint32_t m0 = o[2] | o[4], m1 = o[3] | o[5], mf = o[0] | o[1];   // P0/M0, P1/M1, PF/BL
    const bool pf_first = (ctrlpf & 4) != 0;
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t b0 = byte_masks((m0 >> (4 * k)) & 0xF), b1 = byte_masks((m1 >> (4 * k)) & 0xF);
        const uint32_t bf = byte_masks((mf >> (4 * k)) & 0xF), bp = byte_masks((o[0] >> (4 * k)) & 0xF);
        const uint32_t cfl = pick(bp, cp, cf);   // the playfield's colour where it is set, else the ball's
        const uint32_t v = pf_first ? pick(bf, cfl, pick(b0, c0, pick(b1, c1, cb)))
                                    : pick(b0, c0, pick(b1, c1, pick(bf, cfl, cb)));
        w[k] = v & byte_masks((shown >> (4 * k)) & 0xF);
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

// Row `row` drawn left to right, 16 pixels at a time: the row snapshot, then
// each logged write from its x position on, every write applied once.
// emit(seg, q) receives pixels 16 seg .. 16 seg + 15 packed little-endian.
// The row's first kPre entries are loaded together, before any is needed (one
// memory round trip instead of one per entry); later ones as they come.
constexpr uint32_t kPre = 8;

template <class Pal, class Emit>
__device__ __forceinline__ void render_row(const uint8_t* frame_log, int row, const Pal& pal, Emit&& emit) {
    const uint8_t* rec = frame_log + row * kSnapBytes;
    const uint4 s = *reinterpret_cast<const uint4*>(rec);
    const uint4 s2 = *reinterpret_cast<const uint4*>(rec + 16);
    Regs r;
    unpack(r, s, s2);
    const uint32_t cnt = (s.w >> 24) & kCountMask;
    const uint32_t* ents = reinterpret_cast<const uint32_t*>(frame_log + kSnapArea) + (s2.w & 0xFFFF);
    if (r.outside && cnt == 0) {
        for (int seg = 0; seg < kCols / 16; ++seg) emit(seg, make_uint4(0, 0, 0, 0));
        return;
    }
    // Eight unconditional loads issued back to back: the entry stream holds
    // 5,280 entries and a frame logs at most 5,251, so the words past a row's
    // last entry are still inside the log (their values are never used).
    // They form a queue in eight registers (no indexing, which would put them
    // in scratch memory): q0 is the next entry; popping shifts the others
    // down and loads the entry after them, if the row has one.
    uint32_t q0 = ents[0], q1 = ents[1], q2 = ents[2], q3 = ents[3];
    uint32_t q4 = ents[4], q5 = ents[5], q6 = ents[6], q7 = ents[7];
    uint32_t ei = 0;
    auto next_entry = [&]() -> uint32_t {
        ++ei;
        q0 = q1; q1 = q2; q2 = q3; q3 = q4; q4 = q5; q5 = q6; q6 = q7;
        q7 = ei + (kPre - 1) < cnt ? ents[ei + (kPre - 1)] : 0u;
        return ei < cnt ? q0 : 0u;
    };
    uint32_t e = cnt ? q0 : 0u;
    PlainRow ps;
    plain_row(ps, r, pal);
    for (int seg = 0; seg < kCols / 16; ++seg) {
        const uint32_t x0 = 16u * (uint32_t)seg;
        if (ei < cnt && (e & 0xFF) <= x0) {
            do {                                    // writes that take effect before the segment
                apply(r, e);
                e = next_entry();
            } while (ei < cnt && (e & 0xFF) <= x0);
            plain_row(ps, r, pal);
        }
        uint4 out = make_uint4(0, 0, 0, 0);
        uint32_t start = 0;                         // first pixel of the current run
        for (;;) {
            const bool more = ei < cnt && (e & 0xFF) < x0 + 16;
            const uint32_t end = more ? (e & 0xFF) - x0 : 16;
            const uint4 px = ps.plain ? draw16_row(ps, r, x0) : draw16(r, x0, (uint32_t)row, pal);
            const uint32_t run = ((1u << end) - 1) & ~((1u << start) - 1);
            out.x = pick(byte_masks(run & 0xF), px.x, out.x);
            out.y = pick(byte_masks((run >> 4) & 0xF), px.y, out.y);
            out.z = pick(byte_masks((run >> 8) & 0xF), px.z, out.z);
            out.w = pick(byte_masks((run >> 12) & 0xF), px.w, out.w);
            if (!more) break;
            const uint32_t xe = e & 0xFF;
            while (ei < cnt && (e & 0xFF) == xe) {  // every write at this pixel, in order
                apply(r, e);
                e = next_entry();
            }
            plain_row(ps, r, pal);
            start = end;
        }
        emit(seg, out);
    }
}

// bytewise maximum of two packed 4 x u8 words: the even and the odd bytes
// as two pairs of 16-bit lanes, one packed maximum each
__device__ __forceinline__ uint32_t max4u8(uint32_t a, uint32_t b) {
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    const uint32_t ae = a & 0x00FF00FFu, be = b & 0x00FF00FFu;
    const uint32_t ao = (a >> 8) & 0x00FF00FFu, bo = (b >> 8) & 0x00FF00FFu;
    const u16x2 me = __builtin_elementwise_max(__builtin_bit_cast(u16x2, ae), __builtin_bit_cast(u16x2, be));
    const u16x2 mo = __builtin_elementwise_max(__builtin_bit_cast(u16x2, ao), __builtin_bit_cast(u16x2, bo));
    return __builtin_bit_cast(uint32_t, me) | (__builtin_bit_cast(uint32_t, mo) << 8);
}

constexpr int kSegs = kCols / 16;            // 10 segments per row

// Frames that only go to the frames output (render mode ALL, slots before the
// last two).  grid = (n, n_slots - 2), block 64..512 threads: a thread per
// row draws into an LDS copy of the frame, which the block then writes out
// in whole 16-byte-per-lane runs (rows written by single threads straight to
// HBM leave partial cache lines and double the write traffic).
__global__ void __launch_bounds__(512) k_render_frames(RenderArgs A) {
    __shared__ uint4 s_f[kFrameBytes / 16];
    const uint32_t i = blockIdx.x, slot = blockIdx.y;
    const bool valid = (A.info[i].slots >> slot) & 1;
    uint4* dst = reinterpret_cast<uint4*>(A.frames + ((size_t)i * A.n_slots + slot) * kFrameBytes);
    if (valid) {
        const uint8_t* lg = A.logs + ((size_t)i * A.n_slots + slot) * kFrameLogBytes;
        for (int row = threadIdx.x; row < kRows; row += blockDim.x)
            render_row(lg, row, ColourPal{}, [&](int seg, const uint4 q) { s_f[row * kSegs + seg] = q; });
    }
    __syncthreads();
    for (int c = threadIdx.x; c < kFrameBytes / 16; c += blockDim.x) dst[c] = valid ? s_f[c] : make_uint4(0, 0, 0, 0);
}

// The last two frame slots: frames output (optional) and the observation.
// grid = n, block 64..512 threads.
__global__ void __launch_bounds__(512) k_render_obs(RenderArgs A) {
    __shared__ uint32_t s_m[kFrameBytes / 4];   // max gray of the two frames
    __shared__ uint8_t s_lut[128];
    extern __shared__ uint4 s_f[];               // the frame being drawn, for the frames output: launched
                                                 // with kFrameBytes of dynamic LDS only when A.frames
    const uint32_t i = blockIdx.x;
    if (A.only && A.only[i] == 0) return;        // not one of the positions asked for
    const StepInfo si = A.info[i];
    const bool bad = (si.err & ERR_BAD_ID) != 0;
    const bool want_obs = A.obs && !bad && (A.force_obs || !si.done);
    for (int j = threadIdx.x; j < 128; j += blockDim.x) s_lut[j] = A.gray[j];
    uint8_t* m = reinterpret_cast<uint8_t*>(s_m);
    __syncthreads();
    const int s0 = (int)A.n_slots - 2;
    bool first = true;
    for (int slot = s0 < 0 ? 0 : s0; slot < (int)A.n_slots; ++slot) {
        const bool valid = !bad && ((si.slots >> slot) & 1);
        const uint8_t* lg = A.logs + ((size_t)i * A.n_slots + slot) * kFrameLogBytes;
        uint8_t* dst = A.frames ? A.frames + ((size_t)i * A.n_slots + slot) * kFrameBytes : nullptr;
        if (!valid && !dst) continue;
        for (int row = threadIdx.x; row < kRows; row += blockDim.x) {
            if (!dst) {        // observation only: the row drawn in gray levels straight away
                if (want_obs && valid) {
                    render_row(lg, row, GrayPal{s_lut}, [&](int seg, const uint4 g) {
                        uint4* mq = reinterpret_cast<uint4*>(s_m + (row * kCols + seg * 16) / 4);
                        if (first) {
                            *mq = g;
                        } else {
                            const uint4 o = *mq;
                            *mq = make_uint4(max4u8(o.x, g.x), max4u8(o.y, g.y), max4u8(o.z, g.z), max4u8(o.w, g.w));
                        }
                    });
                }
                continue;
            }
            auto emit = [&](int seg, const uint4 q) {
                s_f[row * kSegs + seg] = q;
                if (want_obs && valid) {
                    const uint32_t wv[4] = {q.x, q.y, q.z, q.w};
                    uint32_t* mrow = s_m + (row * kCols + seg * 16) / 4;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        uint32_t g = 0;
#pragma unroll
                        for (int b = 0; b < 4; ++b) g |= (uint32_t)s_lut[((wv[j] >> (8 * b)) & 0xFF) >> 1] << (8 * b);
                        mrow[j] = first ? g : max4u8(mrow[j], g);
                    }
                }
            };
            if (valid) {
                render_row(lg, row, ColourPal{}, emit);
            } else {
                for (int seg = 0; seg < kSegs; ++seg) emit(seg, make_uint4(0, 0, 0, 0));
            }
        }
        if (want_obs && valid) first = false;
        __syncthreads();
        if (dst) {                            // whole runs to HBM, then the stage is free again
            uint4* d4 = reinterpret_cast<uint4*>(dst);
            for (int c = threadIdx.x; c < kFrameBytes / 16; c += blockDim.x) d4[c] = s_f[c];
            __syncthreads();
        }
    }
    if (!A.obs) return;
    if (bad || (want_obs && first)) {     // no frame to show
        for (int o = threadIdx.x; o < kObsBytes; o += blockDim.x) A.obs[(size_t)i * kObsBytes + o] = 0;
        return;
    }
    if (!want_obs) return;                // the reset kernel writes the cache observation
    // Exact-area 210x160 -> 84x84.  Output rows 2k and 2k+1 cover source rows
    // 5k .. 5k+4 (weights 2,2,1 and 1,2,2 in half rows); output column j covers
    // source columns 40j/21 .. (40j+39)/21, at most three, weighted by their
    // overlap in 1/21 pixels; the total weight is 200.  A work item is one
    // (row pair, column): the column sums of its five source rows, then both
    // outputs (integer sums in another grouping, so the same values).
    for (int w = threadIdx.x; w < (kObs / 2) * kObs; w += blockDim.x) {
        const int k = w / kObs, oj = w - k * kObs;
        const int c0 = (40 * oj) / 21, c1 = (40 * oj + 39) / 21;
        uint32_t wc[3], cc[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int c = c0 + j;
            wc[j] = c <= c1 ? (uint32_t)(min(40 * oj + 40, 21 * c + 21) - max(40 * oj, 21 * c)) : 0u;
            cc[j] = (uint32_t)min(c, kCols - 1);      // a weight-0 column is read in range
        }
        uint32_t s5[5];
#pragma unroll
        for (int r = 0; r < 5; ++r) {
            const uint8_t* src = m + (5 * k + r) * kCols;
            s5[r] = wc[0] * src[cc[0]] + wc[1] * src[cc[1]] + wc[2] * src[cc[2]];
        }
        uint8_t* out = A.obs + (size_t)i * kObsBytes + 2 * k * kObs + oj;
        out[0] = (uint8_t)((2 * s5[0] + 2 * s5[1] + s5[2] + 100) / 200);
        out[kObs] = (uint8_t)((s5[2] + 2 * s5[3] + 2 * s5[4] + 100) / 200);
    }
}

void launch_render_frames(const RenderArgs& a, uint32_t n_front_slots, uint32_t block, hipStream_t s) {
    hipLaunchKernelGGL(k_render_frames, dim3(a.n, n_front_slots), dim3(block), 0, s, a);
}
void launch_render_obs(const RenderArgs& a, uint32_t block, hipStream_t s) {
    // without a frames output the frame copy in LDS is not needed, and twice
    // as many workgroups fit on a compute unit
    hipLaunchKernelGGL(k_render_obs, dim3(a.n), dim3(block), a.frames ? (size_t)kFrameBytes : 0, s, a);
}

}  // namespace vcs
