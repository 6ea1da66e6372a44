// The TIA's objects over 16-pixel segments of a row, from a row snapshot
// (R[0..31]) and the register writes logged inside the row.  Used by the
// render kernels (colours) and by the interpreter's collision scan (which
// objects meet).
//
// Objects (TIA register definitions, with the conventions of this library):
// the playfield (20 bits PF0 D4..D7, PF1 D7..D0, PF2 D0..D7 over 4-pixel
// blocks, the right half repeated or reflected by CTRLPF D0); players of 8
// pixels from GRP (the vertically delayed copy when VDELP D0), reflected by
// REFP D3, in NUSIZ copies (offsets 0/16/32/64) or double / quad width;
// missiles of 1-8 pixels (NUSIZ D4-D5) with the player's copies, shown when
// ENAM D1 is set and RESMP D1 clear; the ball of 1-8 pixels (CTRLPF D4-D5)
// shown when ENABL D1 (or its delayed copy with VDELBL) is set.  Positions
// wrap at 160.  VBLANK D1 and an early HMOVE's blank (pixels 0-7) show
// nothing.
#pragma once

#include "vcs_device.h"

namespace vcs {

// The row's registers as the 8 snapshot words (byte i = R[i]; byte 15, the
// entry count, cleared), kept packed so a thread holds them in 8 registers.
struct Regs {
    uint32_t w[8];
    uint32_t pfm;             // playfield bits 0..19
    bool outside;
};

template <int I>
__device__ __forceinline__ uint32_t rb(const Regs& r) { return (r.w[I >> 2] >> (8 * (I & 3))) & 0xFF; }

__device__ __forceinline__ uint32_t pf_mask(uint32_t pf0, uint32_t pf1, uint32_t pf2) {
    return ((pf0 >> 4) & 0xF) | ((__builtin_bitreverse32(pf1) >> 24) << 4) | ((pf2 & 0xFF) << 12);
}
__device__ __forceinline__ void update_pf(Regs& r) { r.pfm = pf_mask(rb<R_PF0>(r), rb<R_PF1>(r), rb<R_PF2>(r)); }

// a, b: the two halves of a row snapshot
__device__ __forceinline__ void unpack(Regs& r, const uint4 a, const uint4 b) {
    r.w[0] = a.x; r.w[1] = a.y; r.w[2] = a.z; r.w[3] = a.w & 0x00FFFFFFu;
    r.w[4] = b.x; r.w[5] = b.y; r.w[6] = b.z; r.w[7] = b.w;
    r.outside = ((a.w >> 24) & kRowOutside) != 0;
    update_pf(r);
}

template <int K>
__device__ __forceinline__ void set_byte_in(Regs& r, uint32_t sh, uint32_t v) {
    r.w[K] = (r.w[K] & ~(0xFFu << sh)) | (v << sh);
}
__device__ __forceinline__ void set_byte(Regs& r, uint32_t i, uint32_t v) {
    const uint32_t sh = 8 * (i & 3);
    switch (i >> 2) {
    case 0: set_byte_in<0>(r, sh, v); break;
    case 1: set_byte_in<1>(r, sh, v); break;
    case 2: set_byte_in<2>(r, sh, v); break;
    case 3: set_byte_in<3>(r, sh, v); break;
    case 4: set_byte_in<4>(r, sh, v); break;
    case 5: set_byte_in<5>(r, sh, v); break;
    case 6: set_byte_in<6>(r, sh, v); break;
    default: set_byte_in<7>(r, sh, v); break;
    }
}

// Pixels an object moves left on an HMOVE written at colour clock h of its
// line, with motion nibble n (HMxx >> 4).  The strobe is followed by up to 15
// extra motion pulses at clocks h + 4j (j = 1, 2, ...); the object takes the
// first n ^ 8 of them, and a pulse moves it only in horizontal blank: clocks
// 0-67 of a line, 0-75 on the strobe's line when the strobe came before
// clock 68 (which extends that blank and so holds every object 8 pixels
// back).  In closed form: before clock 68, min(n ^ 8, (75 - h) / 4) - 8 (the
// nibble's signed value while h <= 15); from clock 68 on, the pulses from
// j0 = (231 - h) / 4 on fall in the next line's blank: max(0, (n ^ 8) + 1 -
// j0).
__device__ __forceinline__ int32_t hmove_left(uint32_t h, uint32_t n) {
    const int32_t pulses = (int32_t)((n & 15) ^ 8);
    if (h < 68) return min(pulses, (int32_t)((75 - h) >> 2)) - 8;
    return max(0, pulses + 1 - (int32_t)((231 - h) >> 2));
}

// position p moved `left` pixels to the left (-8..15), wrapping at 160
__device__ __forceinline__ uint32_t hm_move(uint32_t p, int32_t left) {
    int32_t q = (int32_t)p - left;
    q += q < 0 ? 160 : 0;
    q -= q >= 160 ? 160 : 0;
    return (uint32_t)q;
}

// one logged write: x | code << 8 | v0 << 16 | v1 << 24
__device__ __forceinline__ void apply(Regs& r, uint32_t e) {
    const uint32_t code = (e >> 8) & 0xFF, v0 = (e >> 16) & 0xFF, v1 = e >> 24;
    if (code == R_END) {
        r.outside = true;
    } else if (code >= R_HMOVE) {   // all five objects by their motion (a logged HMOVE lands in the row: h = x + 68)
        const uint32_t h = (e & 0xFF) + 68;
        set_byte_in<3>(r, 0, hm_move(rb<R_P0X>(r), hmove_left(h, v0)));
        set_byte_in<3>(r, 8, hm_move(rb<R_P1X>(r), hmove_left(h, v0 >> 4)));
        set_byte_in<5>(r, 0, hm_move(rb<R_M0X>(r), hmove_left(h, v1)));
        set_byte_in<5>(r, 8, hm_move(rb<R_M1X>(r), hmove_left(h, v1 >> 4)));
        set_byte_in<5>(r, 16, hm_move(rb<R_BLX>(r), hmove_left(h, code)));
    } else if (code == R_RESMP) {                                   // RESMP0: flags, missile 0 position
        set_byte_in<5>(r, 24, v0);
        set_byte_in<5>(r, 0, v1);
    } else if (code == R_RESMP + 1) {                               // RESMP1: flags 2, missile 1 position
        set_byte_in<6>(r, 0, v0);
        set_byte_in<5>(r, 8, v1);
    } else if (code == R_GRP0) {                                    // GRP1 to its delayed register
        set_byte_in<4>(r, 8, rb<R_GRP1>(r));
        set_byte_in<2>(r, 16, v0);
    } else if (code == R_GRP1) {                                    // GRP0 and ENABL to theirs
        set_byte_in<4>(r, 0, rb<R_GRP0>(r));
        const uint32_t fl = rb<R_FLAGS>(r);
        set_byte_in<5>(r, 24, (fl & ~8u) | ((fl & 4u) << 1));
        set_byte_in<2>(r, 24, v0);
    } else {
        set_byte(r, code, v0);
        if (code >= R_PF0 && code <= R_PF2) update_pf(r);
    }
}

// 16-bit window of a 160-pixel-periodic pattern: `pat` (bit i = pixel
// start + i, `width` <= 32 pixels) starting at `start`, seen from x0
__device__ __forceinline__ uint32_t window16(uint64_t pat, uint32_t width, uint32_t start, uint32_t x0) {
    uint32_t r = start + 160 - x0;       // (start - x0) mod 160
    if (r >= 160) r -= 160;
    uint64_t m = 0;
    if (r < 16) m = pat << r;
    if (r + width > 160) m |= pat >> (160 - r);
    return (uint32_t)m & 0xFFFF;
}

// copies of a player / missile by NUSIZ mode: offsets packed 8 bits each, count
__device__ __forceinline__ uint32_t copy_offsets(uint32_t mode) {
    // mode: 0 {0}, 1 {0,16}, 2 {0,32}, 3 {0,16,32}, 4 {0,64}, 5 {0}, 6 {0,32,64}, 7 {0}
    const uint32_t t[8] = {0x000000u, 0x001000u, 0x002000u, 0x201000u, 0x004000u, 0x000000u, 0x402000u, 0x000000u};
    return t[mode & 7];
}
__device__ __forceinline__ uint32_t copy_count(uint32_t mode) { return (0x13123221u >> (4 * (mode & 7))) & 0xF; }

// window16 for patterns of at most 16 pixels, in 32-bit arithmetic
__device__ __forceinline__ uint32_t window16s(uint32_t pat, uint32_t width, uint32_t start, uint32_t x0) {
    uint32_t r = start + 160 - x0;
    if (r >= 160) r -= 160;
    uint32_t m = 0;
    if (r < 16) m = pat << r;
    if (r + width > 160) m |= pat >> (160 - r);
    return m & 0xFFFF;
}

// player (position, GRP, REFP, NUSIZ) over x0 .. x0+15
__device__ __forceinline__ uint32_t player16(uint32_t pos, uint32_t grp, uint32_t refp, uint32_t nusiz, uint32_t x0) {
    const uint32_t spr = (refp & 8) ? grp : (__builtin_bitreverse32(grp) >> 24);   // bit d = sprite pixel d
    const uint32_t mode = nusiz & 7;
    if (mode == 0) return spr ? window16s(spr, 8, pos, x0) : 0u;   // one copy, normal width
    uint64_t pat = spr;
    uint32_t width = 8;
    if (mode == 5 || mode == 7) {        // double / quad width: every sprite bit over 2 / 4 pixels
        uint64_t p = 0;
        const uint32_t w = mode == 5 ? 2 : 4;
        for (uint32_t d = 0; d < 8; ++d)
            if ((spr >> d) & 1) p |= (((uint64_t)1 << w) - 1) << (w * d);
        pat = p;
        width = 8 * w;
    }
    const uint32_t offs = copy_offsets(mode), n = copy_count(mode);
    uint32_t m = 0;
    for (uint32_t k = 0; k < n; ++k) {
        uint32_t st = pos + ((offs >> (8 * k)) & 0xFF);
        st = st >= 160 ? st - 160 : st;
        m |= window16(pat, width, st, x0);
    }
    return m;
}

// missile (position, enabled, NUSIZ) over x0 .. x0+15
__device__ __forceinline__ uint32_t missile16(uint32_t pos, bool on, uint32_t nusiz, uint32_t x0) {
    if (!on) return 0;
    const uint32_t mode = nusiz & 7, size = 1u << ((nusiz >> 4) & 3);
    const uint32_t offs = copy_offsets(mode), n = (mode == 5 || mode == 7) ? 1u : copy_count(mode);
    uint32_t m = 0;
    for (uint32_t k = 0; k < n; ++k) {
        uint32_t st = pos + ((offs >> (8 * k)) & 0xFF);
        st = st >= 160 ? st - 160 : st;
        m |= window16s((1u << size) - 1, size, st, x0);
    }
    return m;
}

__device__ __forceinline__ uint32_t rev4(uint32_t n) {
    return ((n & 1) << 3) | ((n & 2) << 1) | ((n & 4) >> 1) | ((n & 8) >> 3);
}

// The objects over x0 .. x0+15 (x0 a multiple of 16, so the segment lies in
// one half of the row): o[0] PF, o[1] BL, o[2] P0, o[3] P1, o[4] M0, o[5] M1
// as 16-bit masks; `shown` = pixels drawn at all (not VBLANK, HMOVE blank).
__device__ __forceinline__ void objects16(const Regs& r, uint32_t x0, uint32_t row, uint32_t (&o)[6],
                                          uint32_t& shown) {
    shown = (r.outside || (rb<R_VBLANK>(r) & 2)) ? 0u : 0xFFFFu;
    if (x0 == 0 && rb<R_HMB>(r) == row + 1) shown &= 0xFF00u;
    const bool right = x0 >= 80;
    const uint32_t ctrlpf = rb<R_CTRLPF>(r), flags = rb<R_FLAGS>(r);
    uint32_t n;
    if (!right) n = (r.pfm >> (x0 >> 2)) & 0xF;
    else if (!(ctrlpf & 1)) n = (r.pfm >> ((x0 - 80) >> 2)) & 0xF;
    else n = rev4((r.pfm >> (16 - ((x0 - 80) >> 2))) & 0xF);
    o[0] = ((n & 1) | ((n & 2) << 3) | ((n & 4) << 6) | ((n & 8) << 9)) * 0xF;
    const bool bl_on = (((flags >> 6) & 1) ? (flags >> 3) : (flags >> 2)) & 1;
    const uint32_t bsize = 1u << ((ctrlpf >> 4) & 3);
    o[1] = bl_on ? window16s((1u << bsize) - 1, bsize, rb<R_BLX>(r), x0) : 0u;
    o[2] = player16(rb<R_P0X>(r), ((flags >> 4) & 1) ? rb<R_GRP0_OLD>(r) : rb<R_GRP0>(r), rb<R_REFP0>(r),
                    rb<R_NUSIZ0>(r), x0);
    o[3] = player16(rb<R_P1X>(r), ((flags >> 5) & 1) ? rb<R_GRP1_OLD>(r) : rb<R_GRP1>(r), rb<R_REFP1>(r),
                    rb<R_NUSIZ1>(r), x0);
    o[4] = missile16(rb<R_M0X>(r), (flags & 1) && !((flags >> 7) & 1), rb<R_NUSIZ0>(r), x0);
    o[5] = missile16(rb<R_M1X>(r), ((flags >> 1) & 1) && !(rb<R_FLAGS2>(r) & 1), rb<R_NUSIZ1>(r), x0);
}

// 10-bit mask of the 16-pixel segments that pixels [start, start + width)
// (mod 160, width <= 32) touch
__device__ __forceinline__ uint32_t span_segs(uint32_t start, uint32_t width) {
    const uint32_t end = start + width - 1;
    const uint32_t from = ~((1u << (start >> 4)) - 1);
    if (end < 160) return ((2u << (end >> 4)) - 1) & from;
    return (0x3FFu & from) | ((2u << ((end - 160) >> 4)) - 1);
}

__device__ __forceinline__ uint32_t copies_segs(uint32_t pos, uint32_t mode, uint32_t n, uint32_t width) {
    const uint32_t offs = copy_offsets(mode);
    uint32_t m = 0;
    for (uint32_t k = 0; k < n; ++k) {
        uint32_t st = pos + ((offs >> (8 * k)) & 0xFF);
        st = st >= 160 ? st - 160 : st;
        m |= span_segs(st, width);
    }
    return m;
}

// The segments of a row where two objects can meet under registers r: where
// the extents of two of the players, missiles and ball overlap, or one of
// them overlaps a playfield block that is set.  Every collision pair has a
// player, missile or ball in it, so no latch can be set elsewhere.
__device__ __forceinline__ uint32_t collision_segs(const Regs& r) {
    const uint32_t ctrlpf = rb<R_CTRLPF>(r), flags = rb<R_FLAGS>(r);
    uint32_t m[5];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const uint32_t nus = i ? rb<R_NUSIZ1>(r) : rb<R_NUSIZ0>(r), mode = nus & 7;
        const uint32_t grp = ((flags >> (4 + i)) & 1) ? (i ? rb<R_GRP1_OLD>(r) : rb<R_GRP0_OLD>(r))
                                                     : (i ? rb<R_GRP1>(r) : rb<R_GRP0>(r));
        const uint32_t pw = mode == 5 ? 16u : (mode == 7 ? 32u : 8u);
        m[i] = grp ? copies_segs(i ? rb<R_P1X>(r) : rb<R_P0X>(r), mode, copy_count(mode), pw) : 0u;
        const bool mon = ((flags >> i) & 1) && !(i ? (rb<R_FLAGS2>(r) & 1) : ((flags >> 7) & 1));
        m[2 + i] = mon ? copies_segs(i ? rb<R_M1X>(r) : rb<R_M0X>(r), mode,
                                     (mode == 5 || mode == 7) ? 1u : copy_count(mode), 1u << ((nus >> 4) & 3))
                       : 0u;
    }
    const bool bl_on = (((flags >> 6) & 1) ? (flags >> 3) : (flags >> 2)) & 1;
    m[4] = bl_on ? span_segs(rb<R_BLX>(r), 1u << ((ctrlpf >> 4) & 3)) : 0u;
    uint32_t one = 0, two = 0;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        two |= one & m[i];
        one |= m[i];
    }
    uint32_t pf = 0;                               // segments with a playfield block set
#pragma unroll
    for (int k = 0; k < 5; ++k) pf |= (((r.pfm >> (4 * k)) & 0xF) != 0 ? 1u : 0u) << k;
    if (!(ctrlpf & 1)) {
        pf |= pf << 5;
    } else {
#pragma unroll
        for (int j = 0; j < 5; ++j) pf |= ((pf >> (4 - j)) & 1) << (5 + j);
    }
    return two | (one & pf);
}

// collision latch bits for the pixels in `px` (a 16-bit mask)
__device__ __forceinline__ uint32_t collide16(const uint32_t (&o)[6], uint32_t px) {
    const uint32_t pf = o[0] & px, bl = o[1] & px, p0 = o[2] & px, p1 = o[3] & px, m0 = o[4] & px, m1 = o[5] & px;
    uint32_t cx = 0;
    cx |= (m0 & p1) ? 1u << 1 : 0u;      // CXM0P
    cx |= (m0 & p0) ? 1u << 0 : 0u;
    cx |= (m1 & p0) ? 1u << 3 : 0u;      // CXM1P
    cx |= (m1 & p1) ? 1u << 2 : 0u;
    cx |= (p0 & pf) ? 1u << 5 : 0u;      // CXP0FB
    cx |= (p0 & bl) ? 1u << 4 : 0u;
    cx |= (p1 & pf) ? 1u << 7 : 0u;      // CXP1FB
    cx |= (p1 & bl) ? 1u << 6 : 0u;
    cx |= (m0 & pf) ? 1u << 9 : 0u;      // CXM0FB
    cx |= (m0 & bl) ? 1u << 8 : 0u;
    cx |= (m1 & pf) ? 1u << 11 : 0u;     // CXM1FB
    cx |= (m1 & bl) ? 1u << 10 : 0u;
    cx |= (bl & pf) ? 1u << 13 : 0u;     // CXBLPF
    cx |= (p0 & p1) ? 1u << 15 : 0u;     // CXPPMM
    cx |= (m0 & m1) ? 1u << 14 : 0u;
    return cx;
}

}  // namespace vcs
