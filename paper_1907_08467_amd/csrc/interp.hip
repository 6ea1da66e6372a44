// 6507 interpreter kernel: one lane per env, one wave per ROM-homogeneous tile.
//
// What it computes (paper, Section 3): the "Atari CPU kernel" -- each env's
// CPU runs the cartridge code, updates its 128 B of RAM and the CPU state, and
// passes every TIA register write on to the renderer instead of drawing.
// Here the TIA writes go into a row log (vcs_device.h) only for the frames
// that will be rendered (all frames, or the last two of the step).
//
// Machine conventions (the paper gives none; the public 6502/TIA/RIOT
// definitions plus these readings):
//  * bus: a = addr & $1FFF; a & $1000 cartridge, else a & $80 == 0 TIA,
//    else a & $200 == 0 RAM[a & $7F], else RIOT;
//  * an instruction that starts at cycle t and lasts n cycles performs all its
//    data accesses at cycle t+n-1; opcode/operand fetches happen at t and have
//    no side effects; RMW writes once; no dummy reads;
//  * a TIA write at cycle c takes effect at colour clock 3(c+1); WSYNC written
//    at c resumes the CPU at 76*(c/76+1); a frame ends after the instruction
//    that turns VSYNC bit 1 on; 320 scanlines without that end the frame
//    (FRAME_CAP), as does an undocumented opcode (ILLEGAL);
//  * RIOT timer in closed form: after TIMnT <- v written at cycle w, a read at
//    t sees e = t-w-1: INTIM = v - e/n while e < (v+1)n, then
//    ($FF - (e - (v+1)n)) & $FF with TIMINT bit 7 set;
//  * decimal ADC/SBC follow the NMOS behaviour described by B. Clark
//    ("Decimal Mode", 6502.org, Appendix A).
//
// Dispatch: each loop iteration every running lane fetches its next opcode;
// the wave then executes one opcode at a time for all lanes that share it
// (readfirstlane + compare), so the opcode's decode word is a scalar and the
// addressing-mode and operation switches of the one generic executor are
// scalar branches.  In lockstep (the common case for envs of one ROM) that is
// a single pass.  TIA writes are queued during the pass and applied in one
// shared block afterwards.
#include "tia_draw.h"

namespace vcs {

enum Mn : int {
    ADC, AND, ASL, BCC, BCS, BEQ, BIT, BMI, BNE, BPL, BRK, BVC, BVS, CLC, CLD, CLI, CLV, CMP,
    CPX, CPY, DEC, DEX, DEY, EOR, INC, INX, INY, JMP, JSR, LDA, LDX, LDY, LSR, NOP, ORA, PHA,
    PHP, PLA, PLP, ROL, ROR, RTI, RTS, SBC, SEC, SED, SEI, STA, STX, STY, TAX, TAY, TSX, TXA,
    TXS, TYA,
    SLO, RLA, SRE, RRA, SAX, LAX, DCP, ISC, ANC, ALR, ARR, SBX, LAS,   // undocumented, stable
    ILL
};
enum Md : int { IMP, ACC, IMM, ZP, ZPX, ZPY, ABS, ABX, ABY, IZX, IZY, IND, REL };

struct OpInfo {
    int mn, md, cyc;
    bool pen;   // +1 cycle on an indexed page cross
};

// Decode of the documented opcodes from their aaabbbcc structure.
constexpr OpInfo decode_doc(int op) {
    const int a = op >> 5, b = (op >> 2) & 7, cc = op & 3;
    OpInfo ill{ILL, IMP, 2, false};
    if (cc == 1) {
        const int mns[8] = {ORA, AND, EOR, ADC, STA, LDA, CMP, SBC};
        const int mds[8] = {IZX, ZP, IMM, ABS, IZY, ZPX, ABY, ABX};
        const int rd_cyc[8] = {6, 3, 2, 4, 5, 4, 4, 4};
        const int st_cyc[8] = {6, 3, 0, 4, 6, 4, 5, 5};
        if (mns[a] == STA) {
            if (b == 2) return ill;
            return OpInfo{STA, mds[b], st_cyc[b], false};
        }
        return OpInfo{mns[a], mds[b], rd_cyc[b], b == 4 || b == 6 || b == 7};
    }
    if (cc == 2) {
        const int mns[8] = {ASL, ROL, LSR, ROR, STX, LDX, DEC, INC};
        const int mn = mns[a];
        const bool rmw = (a < 4) || (a >= 6);
        switch (b) {
        case 0: return a == 5 ? OpInfo{LDX, IMM, 2, false} : ill;
        case 1: return OpInfo{mn, ZP, rmw ? 5 : 3, false};
        case 2:
            if (a < 4) return OpInfo{mn, ACC, 2, false};
            if (a == 4) return OpInfo{TXA, IMP, 2, false};
            if (a == 5) return OpInfo{TAX, IMP, 2, false};
            if (a == 6) return OpInfo{DEX, IMP, 2, false};
            return OpInfo{NOP, IMP, 2, false};
        case 3: return OpInfo{mn, ABS, rmw ? 6 : 4, false};
        case 5: return OpInfo{mn, (a == 4 || a == 5) ? ZPY : ZPX, rmw ? 6 : 4, false};
        case 6:
            if (a == 4) return OpInfo{TXS, IMP, 2, false};
            if (a == 5) return OpInfo{TSX, IMP, 2, false};
            return ill;
        case 7:
            if (a == 4) return ill;
            if (a == 5) return OpInfo{LDX, ABY, 4, true};
            return OpInfo{mn, ABX, 7, false};
        default: return ill;
        }
    }
    if (cc == 0) {
        if (b == 4) {
            const int br[8] = {BPL, BMI, BVC, BVS, BCC, BCS, BNE, BEQ};
            return OpInfo{br[a], REL, 2, false};
        }
        if (b == 6) {
            const int fl[8] = {CLC, SEC, CLI, SEI, TYA, CLV, CLD, SED};
            return OpInfo{fl[a], IMP, 2, false};
        }
        if (b == 2) {
            const int st[8] = {PHP, PLP, PHA, PLA, DEY, TAY, INY, INX};
            const int cy[8] = {3, 4, 3, 4, 2, 2, 2, 2};
            return OpInfo{st[a], IMP, cy[a], false};
        }
        if (b == 0) {
            switch (a) {
            case 0: return OpInfo{BRK, IMP, 7, false};
            case 1: return OpInfo{JSR, ABS, 6, false};
            case 2: return OpInfo{RTI, IMP, 6, false};
            case 3: return OpInfo{RTS, IMP, 6, false};
            case 5: return OpInfo{LDY, IMM, 2, false};
            case 6: return OpInfo{CPY, IMM, 2, false};
            case 7: return OpInfo{CPX, IMM, 2, false};
            default: return ill;
            }
        }
        const int mns[8] = {ILL, BIT, JMP, JMP, STY, LDY, CPY, CPX};
        if (b == 1) return (a == 1 || a >= 4) ? OpInfo{mns[a], ZP, 3, false} : ill;
        if (b == 3) {
            if (a == 0) return ill;
            if (a == 2) return OpInfo{JMP, ABS, 3, false};
            if (a == 3) return OpInfo{JMP, IND, 5, false};
            return OpInfo{mns[a], ABS, 4, false};
        }
        if (b == 5) return (a == 4 || a == 5) ? OpInfo{mns[a], ZPX, 4, false} : ill;
        if (b == 7) return a == 5 ? OpInfo{LDY, ABX, 4, true} : ill;
        return ill;
    }
    return ill;
}

// Decode of every opcode: the documented ones, then the stable undocumented
// ones (NMOS unintended-opcode matrix); JAMs and the unstable ANE, LXA, SHA,
// SHX, SHY, TAS stay ILL.
constexpr OpInfo decode(int op) {
    const OpInfo d = decode_doc(op);
    if (d.mn != ILL) return d;
    const int a = op >> 5, b = (op >> 2) & 7, cc = op & 3;
    OpInfo ill{ILL, IMP, 2, false};
    if (cc == 3) {
        const int combo[8] = {SLO, RLA, SRE, RRA, SAX, LAX, DCP, ISC};
        const int mn = combo[a];
        if (b == 2) {                               // immediate column
            const int imm[8] = {ANC, ANC, ALR, ARR, ILL, ILL, SBX, SBC};
            return imm[a] == ILL ? ill : OpInfo{imm[a], IMM, 2, false};
        }
        if (mn == SAX) {
            switch (b) {
            case 0: return OpInfo{SAX, IZX, 6, false};
            case 1: return OpInfo{SAX, ZP, 3, false};
            case 3: return OpInfo{SAX, ABS, 4, false};
            case 5: return OpInfo{SAX, ZPY, 4, false};
            default: return ill;                    // SHA, TAS, SHA: unstable
            }
        }
        if (mn == LAX) {
            switch (b) {
            case 0: return OpInfo{LAX, IZX, 6, false};
            case 1: return OpInfo{LAX, ZP, 3, false};
            case 3: return OpInfo{LAX, ABS, 4, false};
            case 4: return OpInfo{LAX, IZY, 5, true};
            case 5: return OpInfo{LAX, ZPY, 4, false};
            case 6: return OpInfo{LAS, ABY, 4, true};
            default: return OpInfo{LAX, ABY, 4, true};
            }
        }
        const int mds[8] = {IZX, ZP, IMM, ABS, IZY, ZPX, ABY, ABX};
        const int cyc[8] = {8, 5, 2, 6, 8, 6, 7, 7};
        return OpInfo{mn, mds[b], cyc[b], false};
    }
    // NOPs of every width; the rest of the undocumented cc = 0, 1, 2 opcodes
    // are JAMs or unstable
    if (b == 0 && (op == 0x80 || op == 0x82 || op == 0xC2 || op == 0xE2)) return OpInfo{NOP, IMM, 2, false};
    if (op == 0x89) return OpInfo{NOP, IMM, 2, false};
    if (cc == 0 && b == 1 && (a == 0 || a == 2 || a == 3)) return OpInfo{NOP, ZP, 3, false};
    if (op == 0x0C) return OpInfo{NOP, ABS, 4, false};
    if (cc == 0 && b == 5 && a != 4 && a != 5) return OpInfo{NOP, ZPX, 4, false};
    if (cc == 0 && b == 7 && a != 4 && a != 5) return OpInfo{NOP, ABX, 4, true};
    if (cc == 2 && b == 6 && a != 4 && a != 5) return OpInfo{NOP, IMP, 2, false};
    return ill;
}

constexpr bool combo_mn(int mn) {
    return mn == SLO || mn == RLA || mn == SRE || mn == RRA || mn == DCP || mn == ISC;
}

constexpr int op_len(int md) {
    return (md == IMP || md == ACC) ? 1 : (md == ABS || md == ABX || md == ABY || md == IND) ? 3 : 2;
}

// status flags
constexpr uint32_t FC = 0x01, FZ = 0x02, FI = 0x04, FD = 0x08, FB = 0x10, FU = 0x20, FV = 0x40, FN = 0x80;
// per-instruction events
constexpr uint32_t EV_WSYNC = 1, EV_VSYNC = 2;

// Joystick of the 18 actions (ALE order): actions 2..9 and 10..17 are the
// directions UP, RIGHT, LEFT, DOWN, UPRIGHT, UPLEFT, DOWNRIGHT, DOWNLEFT;
// their pressed bits in SWCHA's high nibble (D7 right, D6 left, D5 down,
// D4 up) are packed one byte per direction; 1 and 10..17 hold fire.
constexpr uint64_t kDirBits = 0x60A0509020408010ull;
__device__ __forceinline__ uint32_t joy_pressed(uint32_t a) {
    const uint32_t dir = a >= 10 ? a - 8 : a;
    return dir >= 2 ? (uint32_t)(kDirBits >> (8 * (dir - 2))) & 0xF0u : 0u;
}
__device__ __forceinline__ bool fire_pressed(uint32_t a) { return a == 1 || a >= 10; }

struct Wave {                 // per-workgroup (uniform) data
    const uint8_t* rom;       // the tile's cartridge: its LDS copy, or its HBM slot
    uint8_t* ram;             // LDS, kRamStride bytes per lane
    uint8_t* tia;             // LDS, kTiaStride bytes per lane
    const uint32_t* pre;      // the tile ROM's predecoded words
    CartMap cm;               // its cartridge mapping
    uint32_t track;           // collision latches tracked
};

__device__ __forceinline__ uint32_t cm_kind(const Wave& W) { return W.cm.a & 3; }
__device__ __forceinline__ uint32_t cm_sc(const Wave& W) { return (W.cm.a >> 2) & 1; }
__device__ __forceinline__ uint32_t cm_tf_mask(const Wave& W) { return W.cm.b >> 16; }
__device__ __forceinline__ uint32_t rom_off(const Wave& W, uint32_t bank, uint32_t a) {
    return cart_rom_off(W.cm.a & 3, W.cm.b & 0xFFFF, bank, a);
}
__device__ __forceinline__ uint32_t hotspot(const Wave& W, uint32_t bank, uint32_t a) {
    return cart_hotspot(W.cm.a & 3, W.cm.a >> 8, (W.cm.a >> 4) & 15, bank, a);
}
constexpr int kRamStride = 132;   // 33 dwords: bank-conflict free for equal offsets
constexpr int kTiaStride = 52;    // 13 dwords (R[0..47] + 1): bank-conflict free

struct Cpu {
    uint32_t a, x, y, sp, p, pc, bank;
    uint64_t base;            // absolute cycle of the start of the lane's base line
    uint32_t cyc;             // cycles since `base`
    int32_t fl;               // scanline of the frame's start write, relative to the base line
    uint32_t cap;             // an instruction starting at or after this cycle ends the frame
    uint32_t swcha, inpt4;
    uint32_t vsync, hmp0, hmp1;
    int64_t tbase;            // absolute
    uint32_t tv, tshift;
    uint32_t ev, err;
    uint32_t ac;              // access cycle of the current instruction
    uint32_t tqr0, tqr1, tqr2;     // queued TIA writes: register (scalar when the address is)
    uint32_t tqv0, tqv1, tqv2;     //   and value
    uint32_t tqm;                  //   and the mask of used slots
    uint32_t ram_off, tia_off;
    uint8_t* log;             // current frame's row log, or nullptr
    uint8_t* xram;            // the env's Superchip RAM (in its DevEnv)
    uint32_t slot, slots;     // its slot; slots completed so far
    int32_t open_row;
    uint32_t open_cnt;        // entries logged in the open row
    uint32_t open_base;       // stream index of the open row's first entry
    uint32_t icount;
    uint32_t ucount;          // instructions executed in wave-uniform mode
    int32_t hmb_line;         // line (relative to the base line) an early HMOVE blanked, or -1
    uint32_t cx;              // collision latches (bit 2r+1 / 2r = D7 / D6 of CX register r)
    int32_t cx_row, cx_x;     // the frame's pixels before (row, x) are in cx
    int32_t cx_need;          // >= 0: a latch read needs the pixels through this clock scanned first
    int32_t ptr_memo;         // >= 0: the (zp,X) address / (zp),Y base of the instruction being run
                              // again, fixed by the run that had scanned through its fetch cycle
    uint32_t log_scratch;     // the row log is the collision scratch copy, not a rendered frame
};

__device__ __forceinline__ uint32_t nz(uint32_t p, uint32_t v) {
    return (p & ~(FN | FZ)) | (v & FN) | (v == 0 ? FZ : 0);
}

// Position of colour clock `clk` (relative to the base line) in the frame's
// rows: (row, first pixel after it)
__device__ __forceinline__ bool cx_scanned(const Cpu& c, int32_t clk) {
    const int32_t line = clk / 228, h = clk % 228;
    const int32_t row = line - c.fl - kFirstRow;
    if (row < 0) return true;
    if (row >= kRows) return c.cx_row >= kRows;
    const int32_t x = h >= 68 ? h - 68 + 1 : 0;
    return c.cx_row > row || (c.cx_row == row && c.cx_x >= x);
}

// TIA data read of address a by an access that sees the beam through clock
// `through`.  A latch read (tracked) whose pixels are not all scanned yet
// records that need and reads 0; the per-lane dispatch then scans the row
// log and runs the instruction again.
__device__ __forceinline__ uint32_t tia_read(Cpu& c, const Wave& W, uint32_t a, int32_t through) {
    const uint32_t r = a & 0x0F;
    if (W.track && r < 8) {
        if (!cx_scanned(c, through)) c.cx_need = through;
        return ((c.cx >> (2 * r)) & 3) << 6;
    }
    return r == 0x0C ? c.inpt4 : (r == 0x0D ? 0x80u : 0u);      // untracked latches read 0 here too
}
// The same for an instruction fetch (kernel loop), whose caller has scanned
// the latches through the fetch cycle's pixels first.
__device__ __forceinline__ uint32_t tia_peek(const Cpu& c, const Wave& W, uint32_t a) {
    const uint32_t r = a & 0x0F;
    if (W.track && r < 8) return ((c.cx >> (2 * r)) & 3) << 6;
    return r == 0x0C ? c.inpt4 : (r == 0x0D ? 0x80u : 0u);
}

__device__ __forceinline__ uint32_t riot_read(const Cpu& c, const Wave& W, uint32_t a, uint32_t t) {
    if (!(a & 4)) {
        const uint32_t r = a & 3;
        return r == 0 ? c.swcha : (r == 2 ? 0x0Bu : 0u);
    }
    const int64_t e = (int64_t)(c.base + t) - c.tbase;
    const int64_t lim = (int64_t)(c.tv + 1) << c.tshift;
    // both outcomes computed and masked: no per-lane branch
    const uint32_t m = 0u - (uint32_t)(e >= lim);
    if (a & 1) return m & 0x80u;
    const uint32_t after = (uint32_t)(0xFF - (e - lim)) & 0xFF;
    const uint32_t before = (uint32_t)(c.tv - (uint32_t)(e >> c.tshift)) & 0xFF;
    return (after & m) | (before & ~m);
}

// Superchip RAM window: cartridge offsets $000-$0FF (write port below $080)
__device__ __forceinline__ bool sc_window(const Wave& W, uint32_t a) { return cm_sc(W) && !(a & 0xF00); }

// data read at cycle t (side effects: bank hotspots)
__device__ __forceinline__ uint32_t rd(Cpu& c, const Wave& W, uint32_t addr, uint32_t t) {
    const uint32_t a = addr & 0x1FFF;
    if (a & 0x1000) {
        c.bank = hotspot(W, c.bank, a);
        if (sc_window(W, a)) return (a & 0x80) ? (uint32_t)c.xram[a & 0x7F] : 0u;   // the write port reads 0
        return W.rom[rom_off(W, c.bank, a)];
    }
    if (!(a & 0x80)) return tia_read(c, W, a, 3 * (int32_t)t + 2);   // the access cycle's own pixels too
    if (!(a & 0x200)) return W.ram[c.ram_off + (a & 0x7F)];
    return riot_read(c, W, a, t);
}

// instruction fetch at cycle t, without side effects; the cartridge area
// shows ROM even in the Superchip RAM window
__device__ __forceinline__ uint32_t peek(const Cpu& c, const Wave& W, uint32_t addr, uint32_t t) {
    const uint32_t a = addr & 0x1FFF;
    if (a & 0x1000) return W.rom[rom_off(W, c.bank, a)];
    if (!(a & 0x80)) return tia_peek(c, W, a);
    if (!(a & 0x200)) return W.ram[c.ram_off + (a & 0x7F)];
    return riot_read(c, W, a, t);
}

// zero-page pointer byte, fetched with the instruction at its first cycle:
// RAM, or a TIA read register (a latch read sees the pixels through
// `through`, like a data read)
__device__ __forceinline__ uint32_t zp_fetch(Cpu& c, const Wave& W, uint32_t z, int32_t through) {
    return (z & 0x80) ? (uint32_t)W.ram[c.ram_off + (z & 0x7F)] : tia_read(c, W, z, through);
}

// data write at cycle t; TIA writes are queued in slot K of the instruction
template <int K>
__device__ __forceinline__ void wr(Cpu& c, const Wave& W, uint32_t addr, uint32_t v, uint32_t t) {
    const uint32_t a = addr & 0x1FFF;
    if (a & 0x1000) {
        c.bank = hotspot(W, c.bank, a);
        if (sc_window(W, a) && !(a & 0x80)) c.xram[a & 0x7F] = (uint8_t)v;   // writes to the read port do nothing
    } else if (!(a & 0x80)) {
        if (cm_kind(W) == CART_3F && a <= 0x3F) c.bank = v & cm_tf_mask(W);   // 3F: selects the lower slice
        if (K == 0) { c.tqr0 = a & 0x3F; c.tqv0 = v & 0xFF; }
        if (K == 1) { c.tqr1 = a & 0x3F; c.tqv1 = v & 0xFF; }
        if (K == 2) { c.tqr2 = a & 0x3F; c.tqv2 = v & 0xFF; }
        c.tqm |= 1u << K;
    } else if (!(a & 0x200)) {
        W.ram[c.ram_off + (a & 0x7F)] = (uint8_t)v;
    } else if ((a & 0x14) == 0x14) {     // TIM1T / TIM8T / TIM64T / T1024T
        c.tv = v & 0xFF;
        c.tshift = (0x0A060300u >> (8 * (a & 3))) & 0xFF;   // intervals 1, 8, 64, 1024
        c.tbase = (int64_t)(c.base + t) + 1;
    }
}

template <int K>
__device__ __forceinline__ void push(Cpu& c, const Wave& W, uint32_t v, uint32_t t) {
    wr<K>(c, W, 0x100 | c.sp, v, t);
    c.sp = (c.sp - 1) & 0xFF;
}
__device__ __forceinline__ uint32_t pull(Cpu& c, const Wave& W, uint32_t t) {
    c.sp = (c.sp + 1) & 0xFF;
    return rd(c, W, 0x100 | c.sp, t);
}

__device__ __forceinline__ int32_t sext8(uint32_t v) { return (int32_t)(int8_t)(uint8_t)v; }

__device__ __forceinline__ void do_adc(Cpu& c, uint32_t v) {
    const uint32_t cin = c.p & FC;
    const uint32_t bin = c.a + v + cin;
    if (!(c.p & FD)) {
        const uint32_t ovf = (c.a ^ bin) & (v ^ bin) & 0x80;
        c.p = (c.p & ~(FC | FV)) | (bin > 0xFF ? FC : 0) | (ovf ? FV : 0);
        c.a = bin & 0xFF;
        c.p = nz(c.p, c.a);
        return;
    }
    int32_t lo = (int32_t)((c.a & 0x0F) + (v & 0x0F) + cin);
    if (lo > 9) lo = ((lo + 6) & 0x0F) + 0x10;
    int32_t s = (int32_t)(c.a & 0xF0) + (int32_t)(v & 0xF0) + lo;
    const int32_t ss = sext8(c.a & 0xF0) + sext8(v & 0xF0) + lo;
    if (s >= 0xA0) s += 0x60;
    c.p &= ~(FC | FV | FN | FZ);
    c.p |= (s >= 0x100 ? FC : 0) | ((ss < -128 || ss > 127) ? FV : 0) | (ss & 0x80 ? FN : 0) |
           ((bin & 0xFF) == 0 ? FZ : 0);
    c.a = (uint32_t)s & 0xFF;
}

__device__ __forceinline__ void do_sbc(Cpu& c, uint32_t v) {
    const uint32_t cin = c.p & FC;
    const uint32_t inv = (~v) & 0xFF;
    const uint32_t bin = c.a + inv + cin;
    const uint32_t ovf = (c.a ^ bin) & (inv ^ bin) & 0x80;
    uint32_t res = bin & 0xFF;
    if (c.p & FD) {
        int32_t lo = (int32_t)(c.a & 0x0F) - (int32_t)(v & 0x0F) + (int32_t)cin - 1;
        if (lo < 0) lo = ((lo - 6) & 0x0F) - 0x10;
        int32_t s = (int32_t)(c.a & 0xF0) - (int32_t)(v & 0xF0) + lo;
        if (s < 0) s -= 0x60;
        res = (uint32_t)s & 0xFF;
    }
    c.p = (c.p & ~(FC | FV)) | (bin > 0xFF ? FC : 0) | (ovf ? FV : 0);
    c.p = nz(c.p, bin & 0xFF);
    c.a = res;
}

__device__ __forceinline__ void do_cmp(Cpu& c, uint32_t r, uint32_t v) {
    c.p = (c.p & ~FC) | (r >= v ? FC : 0);
    c.p = nz(c.p, (r - v) & 0xFF);
}

// ARR: (A AND operand) rotated right through C.  Binary: N, Z of the result,
// C = bit 6, V = bit 6 ^ bit 5.  Decimal (NMOS): N = the old C, Z and V from
// the rotate (V: bit 6 changed), then BCD fix-ups of each nibble decided on
// the unrotated value, the high one also giving C.
__device__ __forceinline__ void do_arr(Cpu& c, uint32_t v) {
    const uint32_t t = c.a & v;
    const uint32_t cin = c.p & FC;
    uint32_t r = (t >> 1) | (cin << 7);
    if (!(c.p & FD)) {
        c.p = nz(c.p & ~(FC | FV), r) | ((r >> 6) & 1) | ((((r >> 6) ^ (r >> 5)) & 1) ? FV : 0);
        c.a = r;
        return;
    }
    uint32_t p = c.p & ~(FN | FZ | FV | FC);
    p |= (cin ? FN : 0) | (r == 0 ? FZ : 0) | (((t ^ r) & 0x40) ? FV : 0);
    if ((t & 0x0F) + (t & 0x01) > 5) r = (r & 0xF0) | ((r + 6) & 0x0F);
    if ((t & 0xF0) + (t & 0x10) > 0x50) {
        r = (r + 0x60) & 0xFF;
        p |= FC;
    }
    c.p = p;
    c.a = r;
}

// Decode word of an opcode: mode | mnemonic << 4 | base cycles << 11 |
// page penalty << 15 | length << 16 | reads operand << 18 | writes to ea << 19.
constexpr uint32_t DW_CYC = 11, DW_PEN = 15, DW_LEN = 16, DW_RD = 18, DW_WR = 19;
constexpr uint32_t encode(int op) {
    const OpInfo I = decode(op);
    const bool rmw = I.mn == ASL || I.mn == LSR || I.mn == ROL || I.mn == ROR || I.mn == INC || I.mn == DEC ||
                     combo_mn(I.mn);
    const bool mem = I.md != IMP && I.md != ACC && I.md != REL && I.md != IMM;
    const bool reads = (I.mn == LDA || I.mn == LDX || I.mn == LDY || I.mn == ADC || I.mn == SBC || I.mn == AND ||
                        I.mn == ORA || I.mn == EOR || I.mn == CMP || I.mn == CPX || I.mn == CPY || I.mn == BIT ||
                        I.mn == LAX || I.mn == LAS || I.mn == NOP || rmw) && mem;
    const bool writes = (I.mn == STA || I.mn == STX || I.mn == STY || I.mn == SAX || rmw) && mem;
    return (uint32_t)I.md | ((uint32_t)I.mn << 4) | ((uint32_t)I.cyc << DW_CYC) | ((uint32_t)I.pen << DW_PEN) |
           ((uint32_t)op_len(I.md) << DW_LEN) | ((uint32_t)reads << DW_RD) | ((uint32_t)writes << DW_WR);
}
struct DecodeTable {
    uint32_t w[256];
    constexpr DecodeTable() : w() {
        for (int i = 0; i < 256; ++i) w[i] = encode(i);
    }
};
__constant__ DecodeTable kDecode = DecodeTable();

// Execute one instruction with decode word `d` (wave-uniform) for the lanes
// that fetched it.  Sets c.ac, c.pc, c.cyc (before a WSYNC stall) and queues
// TIA writes.
__device__ __forceinline__ void exec_generic(uint32_t d, Cpu& c, const Wave& W, uint32_t b1, uint32_t b2) {
    const uint32_t md = d & 15, mn = (d >> 4) & 127;
    uint32_t n = (d >> DW_CYC) & 15;
    if (mn == ILL) {
        c.err |= ERR_ILLEGAL;
        return;
    }
    uint32_t ea = 0;
    switch (md) {
    case ZP: ea = b1; break;
    case ZPX: ea = (b1 + c.x) & 0xFF; break;
    case ZPY: ea = (b1 + c.y) & 0xFF; break;
    case ABS: case IND: ea = b1 | (b2 << 8); break;
    case ABX: case ABY: {
        const uint32_t base = b1 | (b2 << 8);
        ea = (base + (md == ABX ? c.x : c.y)) & 0xFFFF;
        if ((d >> DW_PEN) & 1) n += ((base ^ ea) & 0xFF00) ? 1 : 0;
        break;
    }
    case IZX: {
        if (c.ptr_memo >= 0) {
            ea = (uint32_t)c.ptr_memo;
        } else {
            const uint32_t z = (b1 + c.x) & 0xFF;
            const int32_t th = 3 * (int32_t)c.cyc + 2;
            ea = zp_fetch(c, W, z, th) | (zp_fetch(c, W, (z + 1) & 0xFF, th) << 8);
            if (W.track && c.cx_need < 0) c.ptr_memo = (int32_t)ea;   // its latches are final
        }
        break;
    }
    case IZY: {
        uint32_t base;
        if (c.ptr_memo >= 0) {
            base = (uint32_t)c.ptr_memo;
        } else {
            const int32_t th = 3 * (int32_t)c.cyc + 2;
            base = zp_fetch(c, W, b1, th) | (zp_fetch(c, W, (b1 + 1) & 0xFF, th) << 8);
            if (W.track && c.cx_need < 0) c.ptr_memo = (int32_t)base;
        }
        ea = (base + c.y) & 0xFFFF;
        if ((d >> DW_PEN) & 1) n += ((base ^ ea) & 0xFF00) ? 1 : 0;
        break;
    }
    default: break;
    }
    // a pointer taken from latches not scanned yet names no address: stop
    // before any access (the caller scans the log and runs it again).  A
    // pointer that was read keeps its value for the runs that follow (a data
    // access later in the instruction may need the scan carried further,
    // past the pixels the pointer fetch saw).
    if (W.track && c.cx_need >= 0) return;
    const uint32_t next = (c.pc + ((d >> DW_LEN) & 3)) & 0xFFFF;
    uint32_t npc = next;
    if (md == REL) {
        bool taken;
        switch (mn) {
        case BPL: taken = !(c.p & FN); break;
        case BMI: taken = (c.p & FN) != 0; break;
        case BVC: taken = !(c.p & FV); break;
        case BVS: taken = (c.p & FV) != 0; break;
        case BCC: taken = !(c.p & FC); break;
        case BCS: taken = (c.p & FC) != 0; break;
        case BNE: taken = !(c.p & FZ); break;
        default: taken = (c.p & FZ) != 0; break;
        }
        if (taken) {
            const uint32_t tgt = (next + (uint32_t)sext8(b1)) & 0xFFFF;
            n += 1 + (((tgt ^ next) & 0xFF00) ? 1 : 0);
            npc = tgt;
        }
    }
    const uint32_t t = c.cyc + n - 1;     // access cycle
    c.ac = t;
    uint32_t v = b1;                      // operand (immediate, or read below)
    if ((d >> DW_RD) & 1) v = rd(c, W, ea, t);
    uint32_t res = 0;                     // value written to ea when (d >> 17) & 1
    switch (mn) {
    case LDA: c.a = v; c.p = nz(c.p, v); break;
    case LDX: c.x = v; c.p = nz(c.p, v); break;
    case LDY: c.y = v; c.p = nz(c.p, v); break;
    case STA: res = c.a; break;
    case STX: res = c.x; break;
    case STY: res = c.y; break;
    case ADC: do_adc(c, v); break;
    case SBC: do_sbc(c, v); break;
    case AND: c.a &= v; c.p = nz(c.p, c.a); break;
    case ORA: c.a |= v; c.p = nz(c.p, c.a); break;
    case EOR: c.a ^= v; c.p = nz(c.p, c.a); break;
    case CMP: do_cmp(c, c.a, v); break;
    case CPX: do_cmp(c, c.x, v); break;
    case CPY: do_cmp(c, c.y, v); break;
    case BIT: c.p = (c.p & ~(FN | FV | FZ)) | (v & (FN | FV)) | ((c.a & v) == 0 ? FZ : 0); break;
    case ASL: case LSR: case ROL: case ROR: case INC: case DEC: {
        const uint32_t x = md == ACC ? c.a : v;
        const uint32_t ci = c.p & FC;
        uint32_t r, co = ci;
        if (mn == ASL) { r = (x << 1) & 0xFF; co = x >> 7; }
        else if (mn == LSR) { r = x >> 1; co = x & 1; }
        else if (mn == ROL) { r = ((x << 1) | ci) & 0xFF; co = x >> 7; }
        else if (mn == ROR) { r = (x >> 1) | (ci << 7); co = x & 1; }
        else if (mn == INC) { r = (x + 1) & 0xFF; }
        else { r = (x - 1) & 0xFF; }
        c.p = nz((c.p & ~FC) | co, r);
        if (md == ACC) c.a = r;
        res = r;
        break;
    }
    case SLO: case RLA: case SRE: case RRA: case DCP: case ISC: {
        // the shift / rotate / count half; the ALU half follows the write
        const uint32_t ci = c.p & FC;
        uint32_t r, co = ci;
        if (mn == SLO) { r = (v << 1) & 0xFF; co = v >> 7; }
        else if (mn == RLA) { r = ((v << 1) | ci) & 0xFF; co = v >> 7; }
        else if (mn == SRE) { r = v >> 1; co = v & 1; }
        else if (mn == RRA) { r = (v >> 1) | (ci << 7); co = v & 1; }
        else if (mn == DCP) { r = (v - 1) & 0xFF; }
        else { r = (v + 1) & 0xFF; }
        c.p = (c.p & ~FC) | co;
        res = r;
        break;
    }
    case SAX: res = c.a & c.x; break;
    case LAX: c.a = c.x = v; c.p = nz(c.p, v); break;
    case LAS: c.sp &= v; c.a = c.x = c.sp; c.p = nz(c.p, c.a); break;
    case ANC: c.a &= v; c.p = nz(c.p, c.a); c.p = (c.p & ~FC) | (c.a >> 7); break;
    case ALR: c.a &= v; c.p = (c.p & ~FC) | (c.a & 1); c.a >>= 1; c.p = nz(c.p, c.a); break;
    case SBX: {
        const uint32_t t0 = c.a & c.x;
        c.p = (c.p & ~FC) | (t0 >= v ? FC : 0);
        c.x = (t0 - v) & 0xFF;
        c.p = nz(c.p, c.x);
        break;
    }
    case ARR: do_arr(c, v); break;
    case INX: c.x = (c.x + 1) & 0xFF; c.p = nz(c.p, c.x); break;
    case INY: c.y = (c.y + 1) & 0xFF; c.p = nz(c.p, c.y); break;
    case DEX: c.x = (c.x - 1) & 0xFF; c.p = nz(c.p, c.x); break;
    case DEY: c.y = (c.y - 1) & 0xFF; c.p = nz(c.p, c.y); break;
    case TAX: c.x = c.a; c.p = nz(c.p, c.x); break;
    case TAY: c.y = c.a; c.p = nz(c.p, c.y); break;
    case TXA: c.a = c.x; c.p = nz(c.p, c.a); break;
    case TYA: c.a = c.y; c.p = nz(c.p, c.a); break;
    case TSX: c.x = c.sp; c.p = nz(c.p, c.x); break;
    case TXS: c.sp = c.x; break;
    case CLC: c.p &= ~FC; break;
    case SEC: c.p |= FC; break;
    case CLI: c.p &= ~FI; break;
    case SEI: c.p |= FI; break;
    case CLV: c.p &= ~FV; break;
    case CLD: c.p &= ~FD; break;
    case SED: c.p |= FD; break;
    case PHA: push<0>(c, W, c.a, t); break;
    case PHP: push<0>(c, W, c.p | FB | FU, t); break;
    case PLA: c.a = pull(c, W, t); c.p = nz(c.p, c.a); break;
    case PLP: c.p = (pull(c, W, t) & ~FB) | FU; break;
    case JMP:
        if (md == ABS) {
            npc = ea;
        } else {                          // the pointer's high byte stays in its page
            const uint32_t lo = rd(c, W, ea, t);
            const uint32_t hi = rd(c, W, (ea & 0xFF00) | ((ea + 1) & 0xFF), t);
            npc = lo | (hi << 8);
        }
        break;
    case JSR: {
        const uint32_t ret = (next - 1) & 0xFFFF;
        push<0>(c, W, ret >> 8, t);
        push<1>(c, W, ret & 0xFF, t);
        npc = ea;
        break;
    }
    case RTS: {
        const uint32_t lo = pull(c, W, t);
        const uint32_t hi = pull(c, W, t);
        npc = ((lo | (hi << 8)) + 1) & 0xFFFF;
        break;
    }
    case RTI: {
        c.p = (pull(c, W, t) & ~FB) | FU;
        const uint32_t lo = pull(c, W, t);
        const uint32_t hi = pull(c, W, t);
        npc = lo | (hi << 8);
        break;
    }
    case BRK: {
        const uint32_t ret = (c.pc + 2) & 0xFFFF;
        push<0>(c, W, ret >> 8, t);
        push<1>(c, W, ret & 0xFF, t);
        push<2>(c, W, c.p | FB | FU, t);
        c.p |= FI;
        const uint32_t lo = rd(c, W, 0xFFFE, t);
        const uint32_t hi = rd(c, W, 0xFFFF, t);
        npc = lo | (hi << 8);
        break;
    }
    default: break;                       // NOP, branches
    }
    if ((d >> DW_WR) & 1) wr<0>(c, W, ea, res, t);
    if (mn == RRA) do_adc(c, res);        // the ALU half of the undocumented pairs,
    else if (mn == ISC) do_sbc(c, res);   // after the write of their shifted /
    else if (mn == DCP) do_cmp(c, c.a, res);   // counted operand
    else if (mn == SLO) { c.a |= res; c.p = nz(c.p, c.a); }
    else if (mn == RLA) { c.a &= res; c.p = nz(c.p, c.a); }
    else if (mn == SRE) { c.a ^= res; c.p = nz(c.p, c.a); }
    c.pc = npc;
    c.cyc = t + 1;
}

// ------------------------------------------------------------ row log

__device__ __forceinline__ void log_finalize(Cpu& c) {
    if (c.open_row >= 0 && c.open_cnt) c.log[c.open_row * kSnapBytes + 15] = (uint8_t)c.open_cnt;
}

// Take the snapshots of every row up to `target` (inclusive) from the
// registers as they are now; the new rows' entries start where the open
// row's end.
__device__ __forceinline__ void log_advance(Cpu& c, const Wave& W, int32_t target) {
    if (target > kRows - 1) target = kRows - 1;
    while (c.open_row < target) {
        log_finalize(c);
        c.open_row++;
        c.open_base += c.open_cnt;
        c.open_cnt = 0;
        const uint32_t* s = reinterpret_cast<const uint32_t*>(W.tia + c.tia_off);
        uint4* d = reinterpret_cast<uint4*>(c.log + c.open_row * kSnapBytes);
        d[0] = make_uint4(s[0], s[1], s[2], s[3] & 0x00FFFFFFu);
        d[1] = make_uint4(s[4], s[5], s[6], (s[7] & 0xFFFF0000u) | c.open_base);
    }
}

// The entry of a write in the open row.  Every write logs at most one entry
// and a row's count stays within its bound, so the guard (an error bit
// instead of a truncated row) is never expected to fire.
__device__ __forceinline__ void log_entry(Cpu& c, int32_t row, uint32_t x, uint32_t code, uint32_t v0, uint32_t v1) {
    if (row < 0 || row >= kRows) return;
    if (c.open_cnt >= kCountMask || c.open_base + c.open_cnt >= (uint32_t)kFrameEntries) {
        c.err |= ERR_LOG;
        return;
    }
    *reinterpret_cast<uint32_t*>(c.log + kSnapArea + 4 * (c.open_base + c.open_cnt)) =
        x | (code << 8) | (v0 << 16) | (v1 << 24);
    c.open_cnt++;
}

// A render-visible event with effect at colour clock 3(t+1): bring the
// snapshots up to date; if it lands in a row's visible part, log it there.
__device__ __forceinline__ void log_event(Cpu& c, const Wave& W, uint32_t t, uint32_t code, uint32_t v0,
                                          uint32_t v1) {
    const uint32_t ln = (t + 1) / 76;
    const uint32_t h = 3 * (t + 1 - 76 * ln);
    const int32_t row = (int32_t)ln - c.fl - kFirstRow;
    log_advance(c, W, h >= 68 ? row : row - 1);
    if (h >= 68) log_entry(c, row, h - 68, code, v0, v1);
}

// the frame ends with its last cycle at t: rows after it are outside
__device__ __forceinline__ void log_close(Cpu& c, const Wave& W, uint32_t t) {
    log_event(c, W, t, R_END, 0, 0);
    log_finalize(c);
    for (int32_t r = c.open_row + 1; r < kRows; ++r) {
        uint4* d = reinterpret_cast<uint4*>(c.log + r * kSnapBytes);
        d[0] = make_uint4(0, 0, 0, kRowOutside << 24);
        d[1] = make_uint4(0, 0, 0, 0);
    }
    c.log = nullptr;
    if (!c.log_scratch) c.slots |= 1u << c.slot;
}

// ------------------------------------------------------------ collisions

// Latches of the pixels of the frame's rows from the scan position
// (c.cx_row, c.cx_x) up to row_end (pixels of row_end before x_end), from
// the row log: each row's snapshot and logged writes, 16 pixels at a time.
__device__ __forceinline__ void cx_scan(Cpu& c, const Wave& W, int32_t row_end, int32_t x_end) {
    if (row_end > kRows) {
        row_end = kRows;
        x_end = 0;
    }
    // the last whole row this call scanned: a whole row with the same snapshot
    // and the same writes draws the same pixels (unless an HMOVE blank falls
    // on one of the two), so its latch bits are already in c.cx
    uint4 pa = make_uint4(0, 0, 0, 0), pb = make_uint4(0, 0, 0, 0);
    uint32_t pcnt = ~0u;
    const uint32_t* pents = nullptr;
    while (c.cx_row < row_end || (c.cx_row == row_end && c.cx_x < x_end && row_end < kRows)) {
        const int32_t r = c.cx_row;
        const uint32_t xe = r < row_end ? 160u : (uint32_t)x_end;
        const uint8_t* rec = c.log + r * kSnapBytes;
        const uint4 sa = reinterpret_cast<const uint4*>(rec)[0], sb = reinterpret_cast<const uint4*>(rec)[1];
        const uint32_t cnt = r == c.open_row ? c.open_cnt : ((sa.w >> 24) & kCountMask);
        const uint32_t* ents = reinterpret_cast<const uint32_t*>(c.log + kSnapArea) + (sb.w & 0xFFFF);
        const bool whole = c.cx_x == 0 && xe == 160;
        if (whole && cnt == pcnt) {
            const uint32_t hmb = (sb.z >> 8) & 0xFF;
            bool same = sa.x == pa.x && sa.y == pa.y && sa.z == pa.z && ((sa.w ^ pa.w) & 0x80FFFFFFu) == 0 &&
                        sb.x == pb.x && sb.y == pb.y && sb.z == pb.z && ((sb.w ^ pb.w) & 0xFFFF0000u) == 0 &&
                        hmb != (uint32_t)r && hmb != (uint32_t)r + 1;
            for (uint32_t i = 0; same && i < cnt; ++i) same = ents[i] == pents[i];
            if (same) {
                c.cx_row = r + 1;
                continue;
            }
        }
        Regs R;
        unpack(R, sa, sb);
        uint32_t ei = 0, cur = (uint32_t)c.cx_x;
        while (cur < xe) {
            while (ei < cnt && (ents[ei] & 0xFF) <= cur) apply(R, ents[ei++]);
            const uint32_t nx = ei < cnt ? min((uint32_t)(ents[ei] & 0xFF), xe) : xe;
            // only drawn runs, and in them only the segments where two objects can meet
            uint32_t segs = (R.outside || (rb<R_VBLANK>(R) & 2)) ? 0u : collision_segs(R);
            segs &= ((2u << ((nx - 1) >> 4)) - 1) & ~((1u << (cur >> 4)) - 1);
            while (segs) {
                const uint32_t x0 = 16u * (uint32_t)__builtin_ctz(segs);
                segs &= segs - 1;
                uint32_t o[6], shown;
                objects16(R, x0, (uint32_t)r, o, shown);
                const uint32_t lo = cur > x0 ? cur - x0 : 0u, hi = nx < x0 + 16 ? nx - x0 : 16u;
                const uint32_t run = ((1u << hi) - 1) & ~((1u << lo) - 1);
                c.cx |= collide16(o, shown & run);
            }
            cur = nx;
        }
        if (whole) {
            pa = sa;
            pb = sb;
            pcnt = cnt;
            pents = ents;
        } else {
            pcnt = ~0u;
        }
        if (xe == 160) {
            c.cx_row = r + 1;
            c.cx_x = 0;
        } else {
            c.cx_x = (int32_t)xe;
        }
    }
}

// Scan the pixels through colour clock `through` (relative to the base line)
// into the latches; the rows the beam has reached get their snapshots first
// (as the next logged write would take them).  through < 0: the whole frame
// (its log is complete).
__device__ __forceinline__ void cx_catch_up(Cpu& c, const Wave& W, int32_t through) {
    if (through < 0) {
        cx_scan(c, W, kRows, 0);
        return;
    }
    const int32_t line = through / 228, h = through % 228;
    const int32_t row = line - c.fl - kFirstRow;
    if (row < 0) return;
    log_advance(c, W, h >= 68 ? row : row - 1);
    cx_scan(c, W, row, h >= 68 ? h - 68 + 1 : 0);
}

// Position a RESPx (players, +5) or RESMx / RESBL (+4) write at cycle t sets.
__device__ __forceinline__ uint32_t reset_pos(uint32_t t, uint32_t delay) {
    const uint32_t h = 3 * ((t + 1) % 76);
    return h < 68 ? delay - 2 : (h - 68 + delay) % 160;
}

// Full-byte register k (R[32 + k]) shows in R_FLAGS bit k (R_FLAGS2 bit 0
// for k = 8): ENAM0, ENAM1, ENABL, ENABL (delayed), RESMP0, RESMP1 by D1,
// VDELP0, VDELP1, VDELBL by D0.  The flags byte a write of v makes:
__device__ __forceinline__ uint32_t flags_after(const uint8_t* R, uint32_t k, uint32_t v) {
    const uint32_t bit = (k >= 4 && k <= 6) ? (v & 1) : ((v >> 1) & 1);
    return k == 8 ? bit : (R[R_FLAGS] & ~(1u << k)) | (bit << k);
}
__device__ __forceinline__ void set_flag_reg(uint8_t* R, uint32_t k, uint32_t v, uint32_t flags) {
    R[R_ENAM0 + k] = (uint8_t)v;
    R[k == 8 ? R_FLAGS2 : R_FLAGS] = (uint8_t)flags;
}


// Apply one queued TIA write of `v` to register `reg` made at cycle t: the
// row-log entries of what it changes for the renderer, then the registers.
__device__ __forceinline__ void tia_apply(Cpu& c, const Wave& W, uint32_t reg, uint32_t v, uint32_t t) {
    uint8_t* R = W.tia + c.tia_off;
    const bool lg = c.log != nullptr;
    if (W.track && reg == 0x2C) {               // CXCLR: the latches restart at clock 3(t+1)
        const int32_t ln = (int32_t)((t + 1) / 76), h = 3 * ((int32_t)(t + 1) - 76 * ln);
        const int32_t row = ln - c.fl - kFirstRow;
        c.cx = 0;
        if (row < 0) {
            c.cx_row = 0;
            c.cx_x = 0;
        } else if (row >= kRows) {
            c.cx_row = kRows;
            c.cx_x = 0;
        } else if (row > c.cx_row || (row == c.cx_row && h - 68 > c.cx_x)) {
            c.cx_row = row;
            c.cx_x = h >= 68 ? h - 68 : 0;
        }
        return;
    }
    switch (reg) {
    case 0x00:
        if ((v & 2) && !(c.vsync & 2)) c.ev |= EV_VSYNC;
        c.vsync = v;
        return;
    case 0x02: c.ev |= EV_WSYNC; return;
    case 0x20: c.hmp0 = v; return;
    case 0x21: c.hmp1 = v; return;
    case 0x22: case 0x23: case 0x24: R[R_HMM0 + reg - 0x22] = (uint8_t)v; return;
    case 0x2B: c.hmp0 = 0; c.hmp1 = 0; R[R_HMM0] = R[R_HMM1] = R[R_HMBL] = 0; return;
    case 0x1B:                                  // GRP0; GRP1 to its delayed copy
        if (lg) log_event(c, W, t, R_GRP0, v, 0);
        R[R_GRP1_OLD] = R[R_GRP1];
        R[R_GRP0] = (uint8_t)v;
        return;
    case 0x1C:                                  // GRP1; GRP0 and ENABL to their delayed copies
        if (lg) log_event(c, W, t, R_GRP1, v, 0);
        R[R_GRP0_OLD] = R[R_GRP0];
        R[R_GRP1] = (uint8_t)v;
        R[R_ENABL_OLD] = R[R_ENABL];
        R[R_FLAGS] = (uint8_t)((R[R_FLAGS] & ~8u) | ((R[R_FLAGS] & 4u) << 1));
        return;
    case 0x1D: case 0x1E: case 0x1F: case 0x25: case 0x26: case 0x27: {
        // (every entry is logged before the registers change: logging first
        // takes the snapshots of the rows before the write)
        const uint32_t k = reg <= 0x1F ? reg - 0x1D : reg - 0x25 + 4;
        const uint32_t fl = flags_after(R, k, v);
        if (lg) log_event(c, W, t, R_FLAGS, fl, 0);
        set_flag_reg(R, k, v, fl);
        return;
    }
    case 0x28: case 0x29: {                     // RESMP: the release puts the missile at the player's centre
        const uint32_t i = reg - 0x28;
        const uint32_t was = (R[R_RESMP0 + i] >> 1) & 1;
        const uint32_t fl = flags_after(R, 7 + i, v);
        const bool release = !(v & 2) && was;
        const uint32_t mode = R[R_NUSIZ0 + i] & 7;
        const uint32_t pos = (R[R_P0X + i] + (mode == 5 ? 6u : mode == 7 ? 10u : 3u)) % 160;
        if (lg) log_event(c, W, t, R_RESMP + i, fl, release ? pos : R[R_M0X + i]);
        if (release) R[R_M0X + i] = (uint8_t)pos;
        set_flag_reg(R, 7 + i, v, fl);
        return;
    }
    case 0x2A: {                                // HMOVE: every object by the pulses its blank takes, now
        const uint32_t ln = (t + 1) / 76, h = 3 * (t + 1 - 76 * ln);
        const uint32_t p0 = hm_move(R[R_P0X], hmove_left(h, c.hmp0 >> 4));
        const uint32_t p1 = hm_move(R[R_P1X], hmove_left(h, c.hmp1 >> 4));
        const uint32_t m0 = hm_move(R[R_M0X], hmove_left(h, R[R_HMM0] >> 4));
        const uint32_t m1 = hm_move(R[R_M1X], hmove_left(h, R[R_HMM1] >> 4));
        const uint32_t bl = hm_move(R[R_BLX], hmove_left(h, R[R_HMBL] >> 4));
        if (lg)   // one entry: the renderer applies the five motion nibbles itself
            log_event(c, W, t, R_HMOVE | ((R[R_HMBL] >> 4) & 15), ((c.hmp0 >> 4) & 15) | (c.hmp1 & 0xF0),
                      ((R[R_HMM0] >> 4) & 15) | (R[R_HMM1] & 0xF0));
        R[R_P0X] = (uint8_t)p0; R[R_P1X] = (uint8_t)p1;
        R[R_M0X] = (uint8_t)m0; R[R_M1X] = (uint8_t)m1; R[R_BLX] = (uint8_t)bl;
        if (h < 68) {                           // written in the horizontal blank: pixels 0-7 of the line blank
            c.hmb_line = (int32_t)ln;
            const int32_t row = (int32_t)ln - c.fl - kFirstRow;
            if (row >= 0 && row < kRows) R[R_HMB] = (uint8_t)(row + 1);
        }
        return;
    }
    default: break;
    }
    uint32_t code, v0 = v;
    if (reg >= 0x06 && reg <= 0x0F) code = reg - 0x06;
    else if (reg == 0x01) code = R_VBLANK;
    else if (reg == 0x04 || reg == 0x05) code = R_NUSIZ0 + (reg - 0x04);
    else if (reg == 0x10 || reg == 0x11) {
        code = R_P0X + (reg - 0x10);
        v0 = reset_pos(t, 5);
    } else if (reg >= 0x12 && reg <= 0x14) {
        code = R_M0X + (reg - 0x12);
        v0 = reset_pos(t, 4);
    } else {
        return;   // audio and the rest: no emulated effect
    }
    if (lg) log_event(c, W, t, code, v0, 0);
    R[code] = (uint8_t)v0;
}

__device__ __forceinline__ void apply_queue(Cpu& c, const Wave& W, uint32_t t) {
    if (c.tqm) {
        if (c.tqm & 1) tia_apply(c, W, c.tqr0, c.tqv0, t);
        if (c.tqm & 2) tia_apply(c, W, c.tqr1, c.tqv1, t);
        if (c.tqm & 4) tia_apply(c, W, c.tqr2, c.tqv2, t);
    }
}

__device__ __forceinline__ uint32_t rfl(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ uint32_t rdl(uint32_t v, int lane) { return (uint32_t)__builtin_amdgcn_readlane((int)v, lane); }
__device__ __forceinline__ int32_t rdl(int32_t v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
__device__ __forceinline__ int32_t rfl(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// ------------------------------------------------------- wave-uniform path
//
// When every running lane of the wave is at the same PC, bank, cycle, frame
// line and row-log position, those stay in scalar registers: one scalar load
// of the predecoded ROM gives opcode, operands and decode word, addressing
// and timing run on the scalar unit, and only the data (A, X, Y, P, SP, RAM,
// TIA registers, log stores) is per lane.  Branches whose outcome differs,
// page-crossing penalties or stack targets that differ, and frames that end
// in some lanes only hand the wave back to the per-lane path; so do the
// instructions this path does not cover (indirect modes, JMP (ind), RTI, BRK,
// indexed accesses outside RAM/cartridge), which the per-lane path executes.
struct Fast {
    uint32_t pc, bank, cyc, cap, orow, ocnt, obase;
    int32_t fl;
    uint32_t logon;
    uint32_t partial;   // 1: other running lanes are elsewhere; stop at the next line start
    uint32_t stop;
    uint32_t lim;       // cap, or 0 once the run must stop: one compare ends the run for either
};

__device__ __forceinline__ bool all_lanes(bool p) { return __builtin_amdgcn_ballot_w64(!p) == 0; }

// Stores the scalar path leaves to the per-lane path: VSYNC (it may end the
// frame), the motion registers, HMOVE, HMCLR, RESMP, CXCLR and timer writes.
// Keeping them out leaves the per-lane VSYNC, motion, collision and timer
// state untouched inside the scalar loop.
__device__ __forceinline__ bool tia_exit_reg(uint32_t reg) {
    return reg == 0x00 || (reg >= 0x20 && reg <= 0x24) || reg == 0x28 || reg == 0x29 || reg == 0x2A || reg == 0x2B ||
           reg == 0x2C;
}
__device__ __forceinline__ uint32_t fast_store_ok(uint32_t a) {
    if (a & 0x1000) return 1;                             // cartridge: bank hotspots only
    if (!(a & 0x80)) return tia_exit_reg(a & 0x3F) ? 0u : 1u;   // TIA
    if (!(a & 0x200)) return 1;                           // RAM
    return (a & 0x14) != 0x14 ? 1u : 0u;                  // RIOT: everything but the timer
}

// Store classes of a static address, kept in the predecoded ROM word of a
// store instruction (its byte 3) so the scalar path needs no address decode.
constexpr uint32_t SC_RAM = 0, SC_WSYNC = 1, SC_IGNORE = 2, SC_EXIT = 3, SC_CART = 4, SC_TIA = 0x20;
// SC_TIA | code: a register stored as is; SC_TIAS | code: a position from
// the cycle or a flags byte; SC_TIAG | code: GRP0 / GRP1 (the delayed copies)
constexpr uint32_t SC_TIAS = 0x40, SC_TIAG = 0x60;
// predecoded classes that depend on the cartridge: an absolute access to the
// Superchip RAM window, and a 3F slice-select store to an ignored TIA register
constexpr uint32_t SC_XRAM = 5, SC_3F = 6;
// TIA store codes past the snapshot registers: ENAM0, ENAM1, ENABL, VDELP0,
// VDELP1, VDELBL (SC_TIAS | kScFlag0 + i), written as their full byte and a
// new flags byte
constexpr uint32_t kScFlag0 = 26;

// Class of a store to a (13 bits): RAM, WSYNC, a TIA register the scalar path
// writes (SC_TIA, SC_TIAS or SC_TIAG | its code), a write that changes nothing emulated, a
// cartridge access, or one the scalar path leaves to the per-lane path
// (fast_store_ok).
__device__ __forceinline__ uint32_t store_class(uint32_t a) {
    if (a & 0x1000) return SC_CART;
    if (!(a & 0x80)) {
        const uint32_t reg = a & 0x3F;
        if (reg == 0x02) return SC_WSYNC;
        if (tia_exit_reg(reg)) return SC_EXIT;
        if (reg >= 0x06 && reg <= 0x0F) return SC_TIA | (reg - 0x06);
        if (reg == 0x01) return SC_TIA | R_VBLANK;
        if (reg == 0x04 || reg == 0x05) return SC_TIA | (R_NUSIZ0 + reg - 0x04);
        if (reg == 0x1B) return SC_TIAG | R_GRP0;
        if (reg == 0x1C) return SC_TIAG | R_GRP1;
        if (reg == 0x10 || reg == 0x11) return SC_TIAS | (R_P0X + reg - 0x10);
        if (reg >= 0x12 && reg <= 0x14) return SC_TIAS | (R_M0X + reg - 0x12);
        if (reg >= 0x1D && reg <= 0x1F) return SC_TIAS | (kScFlag0 + reg - 0x1D);
        if (reg >= 0x25 && reg <= 0x27) return SC_TIAS | (kScFlag0 + 3 + reg - 0x25);
        return SC_IGNORE;   // audio and the rest
    }
    if (!(a & 0x200)) return SC_RAM;
    return (a & 0x14) == 0x14 ? SC_EXIT : SC_IGNORE;
}

// Write of per-lane value v to TIA register class `sc` (SC_TIA/S/G | code) at
// scalar cycle t, with its row-log entry.  The scalar path takes the colour,
// playfield, control, reflection, VBLANK and NUSIZ registers, the object
// resets, the players' graphics and the enable and vertical-delay bits
// (logged as the new flags byte); motion, HMOVE, RESMP and CXCLR go to the
// per-lane path.  A GRP0 / GRP1 entry also stands for the copy to the delayed
// registers (the other player's graphics; with GRP1, ENABL), which the
// renderer repeats from its own state.  Returns 0, before changing anything,
// when the row's entries are full (the per-lane path then records the error).
// PLAIN 1: `sc` is known to be SC_TIA | code (a register stored as is); the
// code may then differ between lanes.  PLAIN 2: `sc` is SC_TIA or SC_TIAG |
// code (no object reset, enable or vertical-delay register).
template <int PLAIN = 0>
__device__ __forceinline__ uint32_t fast_tia_code(Cpu& c, const Wave& W, Fast& F, uint32_t sc, uint32_t v,
                                                  uint32_t t) {
    const uint32_t ln = (t + 1) / 76;
    const uint32_t h = 3 * (t + 1 - 76 * ln);
    uint8_t* R = W.tia + c.tia_off;
    uint32_t code = sc & 0x1F;
    uint32_t v0 = v, full = 0;
    if (PLAIN == 0 && sc >= SC_TIAS && sc < SC_TIAG) {
        if (code == R_P0X || code == R_P1X) {
            v0 = h < 68 ? 3u : (h - 68 + 5) % 160;
        } else if (code >= R_M0X && code <= R_BLX) {
            v0 = h < 68 ? 2u : (h - 68 + 4) % 160;
        } else if (code >= kScFlag0) {       // ENAM0/1, ENABL (D1), VDELP0/1, VDELBL (D0)
            const uint32_t i = code - kScFlag0;
            const uint32_t k = i < 3 ? i : i + 1;
            const uint32_t bit = i < 3 ? (v >> 1) & 1 : v & 1;
            v0 = (R[R_FLAGS] & ~(1u << k)) | (bit << k);
            full = R_ENAM0 + k;
            code = R_FLAGS;
        }
    }
    if (F.logon) {
        // rows before the one the write lands in (its own row too when the
        // write lands in the visible part) get their snapshots first
        const int32_t row = (int32_t)ln - F.fl - kFirstRow;
        const int32_t vis = h >= 68 ? 1 : 0;
        int32_t target = row - 1 + vis;
        target = target > kRows - 1 ? kRows - 1 : target;
        if ((int32_t)F.orow <= target) {
            if (F.orow > 0) {
                if (F.ocnt) c.log[(F.orow - 1) * kSnapBytes + 15] = (uint8_t)F.ocnt;
            }
            F.obase += F.ocnt;       // the new rows' entries start after the open row's
            F.ocnt = 0;
            const uint32_t* src = reinterpret_cast<const uint32_t*>(R);
            const uint4 snap0 = make_uint4(src[0], src[1], src[2], src[3] & 0x00FFFFFFu);
            const uint4 snap1 = make_uint4(src[4], src[5], src[6], (src[7] & 0xFFFF0000u) | F.obase);
            do {    // F.orow holds the open row + 1 (0 = none)
                uint4* d = reinterpret_cast<uint4*>(c.log + F.orow * kSnapBytes);
                d[0] = snap0;
                d[1] = snap1;
                F.orow++;
            } while ((int32_t)F.orow <= target);
        }
        if (vis) {
            if ((uint32_t)row < (uint32_t)kRows) {
                // the row is the open one here; past the guard the per-lane path records the error
                if (F.ocnt >= kCountMask || F.obase + F.ocnt >= (uint32_t)kFrameEntries) return 0;
                *reinterpret_cast<uint32_t*>(c.log + kSnapArea + 4 * (F.obase + F.ocnt)) =
                    (h - 68) | (code << 8) | (v0 << 16);
                F.ocnt++;
            }
        }
    }
    if (PLAIN != 1 && sc >= SC_TIAG) {
        if (code == R_GRP0) {
            R[R_GRP1_OLD] = R[R_GRP1];
        } else {
            R[R_GRP0_OLD] = R[R_GRP0];
            R[R_ENABL_OLD] = R[R_ENABL];
            R[R_FLAGS] = (uint8_t)((R[R_FLAGS] & ~8u) | ((R[R_FLAGS] & 4u) << 1));
        }
    } else if (full) {
        R[full] = (uint8_t)v;
    }
    R[code] = (uint8_t)v0;
    return 1;
}

// TIA write of per-lane `v` to scalar register `reg` at scalar cycle t (a
// register fast_store_ok accepts).  Sets `wsync`.  Returns 0 when the
// per-lane path must take the write (a full row log).
__device__ __forceinline__ uint32_t fast_tia(Cpu& c, const Wave& W, Fast& F, uint32_t reg, uint32_t v, uint32_t t,
                                             uint32_t& wsync) {
    const uint32_t sc = store_class(reg);
    if (sc == SC_WSYNC) {
        wsync = 1;
        return 1;
    }
    if (sc < SC_TIA) return 1;
    return fast_tia_code(c, W, F, sc, v, t);
}

// Read of scalar address a (13 bits) at scalar cycle t.
__device__ __forceinline__ uint32_t fast_rd(Cpu& c, const Wave& W, Fast& F, uint32_t a, uint32_t t) {
    if (a & 0x1000) {
        F.bank = hotspot(W, F.bank, a);
        return W.rom[rom_off(W, F.bank, a)];
    }
    if (!(a & 0x80)) {
        const uint32_t r = a & 0x0F;
        return r == 0x0C ? c.inpt4 : (r == 0x0D ? 0x80u : 0u);
    }
    if (!(a & 0x200)) return W.ram[c.ram_off + (a & 0x7F)];
    return riot_read(c, W, a, t);
}

// Write of per-lane v to scalar address a (fast_store_ok) at scalar cycle t.
// Returns false when the per-lane path must take the instruction.
__device__ __forceinline__ uint32_t fast_wr(Cpu& c, const Wave& W, Fast& F, uint32_t a, uint32_t v, uint32_t t,
                                            uint32_t& wsync) {
    if (a & 0x1000) {
        F.bank = hotspot(W, F.bank, a);
        return 1;
    }
    if (!(a & 0x80)) return fast_tia(c, W, F, a & 0x3F, v & 0xFF, t, wsync);
    if (!(a & 0x200)) W.ram[c.ram_off + (a & 0x7F)] = (uint8_t)v;
    return 1;   // other RIOT writes (ports) change nothing emulated
}

// Decimal mode of the lanes in exec for ADC/SBC: 0 all binary, 1 all
// decimal, 2 mixed (the per-lane path then takes the instruction).  Keeping
// the choice uniform keeps the scalar loop free of per-lane branches.
__device__ __forceinline__ uint32_t dec_mode(const Cpu& c) {
    const uint64_t d = __builtin_amdgcn_ballot_w64((c.p & FD) != 0);
    if (d == 0) return 0;
    return d == __builtin_amdgcn_ballot_w64(true) ? 1u : 2u;
}

__device__ __forceinline__ void adc_bin(Cpu& c, uint32_t v) {
    const uint32_t bin = c.a + v + (c.p & FC);
    const uint32_t ovf = (c.a ^ bin) & (v ^ bin) & 0x80;
    c.p = (c.p & ~(FC | FV)) | (bin > 0xFF ? FC : 0) | (ovf ? FV : 0);
    c.a = bin & 0xFF;
    c.p = nz(c.p, c.a);
}

// the decimal ADC and SBC of the per-lane path, for lanes known to be in
// decimal mode (their arithmetic compiles to selects)
__device__ __forceinline__ void adc_dec(Cpu& c, uint32_t v) {
    const uint32_t cin = c.p & FC;
    const uint32_t bin = c.a + v + cin;
    int32_t lo = (int32_t)((c.a & 0x0F) + (v & 0x0F) + cin);
    lo = lo > 9 ? ((lo + 6) & 0x0F) + 0x10 : lo;
    int32_t sum = (int32_t)(c.a & 0xF0) + (int32_t)(v & 0xF0) + lo;
    const int32_t ss = sext8(c.a & 0xF0) + sext8(v & 0xF0) + lo;
    sum = sum >= 0xA0 ? sum + 0x60 : sum;
    c.p = (c.p & ~(FC | FV | FN | FZ)) | (sum >= 0x100 ? FC : 0) | ((ss < -128 || ss > 127) ? FV : 0) |
          (ss & 0x80 ? FN : 0) | ((bin & 0xFF) == 0 ? FZ : 0);
    c.a = (uint32_t)sum & 0xFF;
}

__device__ __forceinline__ void sbc_any(Cpu& c, uint32_t v, uint32_t dec) {
    const uint32_t cin = c.p & FC;
    const uint32_t inv = (~v) & 0xFF;
    const uint32_t bin = c.a + inv + cin;
    const uint32_t ovf = (c.a ^ bin) & (inv ^ bin) & 0x80;
    uint32_t res = bin & 0xFF;
    if (dec) {
        int32_t lo = (int32_t)(c.a & 0x0F) - (int32_t)(v & 0x0F) + (int32_t)cin - 1;
        lo = lo < 0 ? ((lo - 6) & 0x0F) - 0x10 : lo;
        int32_t d = (int32_t)(c.a & 0xF0) - (int32_t)(v & 0xF0) + lo;
        d = d < 0 ? d - 0x60 : d;
        res = (uint32_t)d & 0xFF;
    }
    c.p = (c.p & ~(FC | FV)) | (bin > 0xFF ? FC : 0) | (ovf ? FV : 0);
    c.p = nz(c.p, bin & 0xFF);
    c.a = res;
}

// Per-lane ALU part of the read-class operations (operand v); `dm` is the
// uniform decimal mode (dec_mode) for ADC and SBC.
__device__ __forceinline__ void fast_alu(Cpu& c, uint32_t mn, uint32_t v, uint32_t dm = 0) {
    switch (mn) {
    case LDA: c.a = v; c.p = nz(c.p, v); break;
    case LDX: c.x = v; c.p = nz(c.p, v); break;
    case LDY: c.y = v; c.p = nz(c.p, v); break;
    case ADC: if (dm) adc_dec(c, v); else adc_bin(c, v); break;
    case SBC: sbc_any(c, v, dm); break;
    case AND: c.a &= v; c.p = nz(c.p, c.a); break;
    case ORA: c.a |= v; c.p = nz(c.p, c.a); break;
    case EOR: c.a ^= v; c.p = nz(c.p, c.a); break;
    case CMP: do_cmp(c, c.a, v); break;
    case CPX: do_cmp(c, c.x, v); break;
    case CPY: do_cmp(c, c.y, v); break;
    default: c.p = (c.p & ~(FN | FV | FZ)) | (v & (FN | FV)) | ((c.a & v) == 0 ? FZ : 0); break;   // BIT
    }
}

__device__ __forceinline__ uint32_t fast_rmw(Cpu& c, uint32_t mn, uint32_t x) {
    const uint32_t ci = c.p & FC;
    uint32_t r, co = ci;
    if (mn == ASL) { r = (x << 1) & 0xFF; co = x >> 7; }
    else if (mn == LSR) { r = x >> 1; co = x & 1; }
    else if (mn == ROL) { r = ((x << 1) | ci) & 0xFF; co = x >> 7; }
    else if (mn == ROR) { r = (x >> 1) | (ci << 7); co = x & 1; }
    else if (mn == INC) { r = (x + 1) & 0xFF; }
    else { r = (x - 1) & 0xFF; }
    c.p = nz((c.p & ~FC) | co, r);
    return r;
}

// Outcome of one instruction on the wave-uniform path.
enum : uint32_t {
    FS_NEXT = 0,     // executed; F holds the next pc and cycle
    FS_EXIT = 1,     // not executed: the per-lane path takes this instruction
    FS_LANE = 2      // executed; lanes parted, c.pc / c.cyc hold each lane's
};

constexpr bool read_mn(int mn) {
    return mn == LDA || mn == LDX || mn == LDY || mn == ADC || mn == SBC || mn == AND || mn == ORA || mn == EOR ||
           mn == CMP || mn == CPX || mn == CPY || mn == BIT;
}
constexpr bool store_mn(int mn) { return mn == STA || mn == STX || mn == STY; }
constexpr bool rmw_mn(int mn) { return mn == ASL || mn == LSR || mn == ROL || mn == ROR || mn == INC || mn == DEC; }

template <int MN>
__device__ __forceinline__ uint32_t store_value(const Cpu& c) {
    return MN == STA ? c.a : (MN == STX ? c.x : c.y);
}

// End of an instruction that may have written a TIA register: next pc and
// cycle (a WSYNC write stalls to the next line start).
__device__ __forceinline__ uint32_t fast_finish(Fast& F, uint32_t next, uint32_t t, uint32_t wsync) {
    F.pc = next;
    F.cyc = wsync ? 76 * (t / 76 + 1) : t + 1;
    const uint32_t s = wsync & F.partial;
    F.stop = s;
    F.lim &= s - 1u;
    return FS_NEXT;
}

// One instruction with opcode OP (a compile-time constant, so addressing
// mode, operation and base cycles are folded) for every lane in exec;
// TRACK: collision latches tracked.  HOT: run from the hot loop, so the
// instruction is unmarked (it and a branch target stay inside the bank's
// window, and the pc needs no 16-bit wrap).
template <int OP, bool TRACK, bool HOT = false>
__device__ __forceinline__ uint32_t fop(Cpu& c, const Wave& W, Fast& F, uint32_t b1, uint32_t b2, uint32_t aux) {
    constexpr OpInfo I = decode(OP);
    constexpr int MD = I.md, MN = I.mn;
    constexpr uint32_t N = (uint32_t)I.cyc;
    constexpr uint32_t kPcMask = HOT ? 0xFFFFFFFFu : 0xFFFFu;
    const uint32_t next = (F.pc + (uint32_t)op_len(MD)) & kPcMask;
    if constexpr (MN == ILL || MN == BRK || MN == RTI || MD == IZX || MD == IZY || MD == IND || MN >= SLO ||
                  (MN == NOP && MD != IMP)) {
        return FS_EXIT;   // left to the per-lane path (undocumented opcodes included)
    } else if constexpr (MD == IMM) {
        uint32_t dm = 0;
        if constexpr (MN == ADC || MN == SBC) {
            dm = dec_mode(c);
            if (dm == 2) return FS_EXIT;
        }
        fast_alu(c, MN, b1, dm);
        F.pc = next;
        F.cyc += N;
        return FS_NEXT;
    } else if constexpr (MD == ACC) {
        c.a = fast_rmw(c, MN, c.a);
        F.pc = next;
        F.cyc += N;
        return FS_NEXT;
    } else if constexpr (MD == IMP) {
        if constexpr (MN == PHA || MN == PHP) {
            if (!all_lanes(c.sp >= 0x80)) return FS_EXIT;
            W.ram[c.ram_off + (c.sp & 0x7F)] = (uint8_t)(MN == PHA ? c.a : (c.p | FB | FU));
            c.sp = (c.sp - 1) & 0xFF;
        } else if constexpr (MN == PLA || MN == PLP) {
            if (!all_lanes(c.sp >= 0x7F && c.sp <= 0xFE)) return FS_EXIT;
            c.sp = (c.sp + 1) & 0xFF;
            const uint32_t v = W.ram[c.ram_off + (c.sp & 0x7F)];
            if constexpr (MN == PLA) {
                c.a = v;
                c.p = nz(c.p, v);
            } else {
                c.p = (v & ~FB) | FU;
            }
        } else if constexpr (MN == RTS) {
            if (!all_lanes(c.sp >= 0x7F && c.sp <= 0xFD)) return FS_EXIT;
            const uint32_t lo = W.ram[c.ram_off + ((c.sp + 1) & 0x7F)];
            const uint32_t hi = W.ram[c.ram_off + ((c.sp + 2) & 0x7F)];
            c.sp = (c.sp + 2) & 0xFF;
            const uint32_t tgt = ((lo | (hi << 8)) + 1) & 0xFFFF;
            const uint32_t t0 = rfl(tgt);
            if (!all_lanes(tgt == t0)) {
                c.pc = tgt;
                c.cyc = F.cyc + N;
                return FS_LANE;
            }
            F.pc = t0;
            F.cyc += N;
            return FS_NEXT;
        } else if constexpr (MN == INX) { c.x = (c.x + 1) & 0xFF; c.p = nz(c.p, c.x); }
        else if constexpr (MN == INY) { c.y = (c.y + 1) & 0xFF; c.p = nz(c.p, c.y); }
        else if constexpr (MN == DEX) { c.x = (c.x - 1) & 0xFF; c.p = nz(c.p, c.x); }
        else if constexpr (MN == DEY) { c.y = (c.y - 1) & 0xFF; c.p = nz(c.p, c.y); }
        else if constexpr (MN == TAX) { c.x = c.a; c.p = nz(c.p, c.x); }
        else if constexpr (MN == TAY) { c.y = c.a; c.p = nz(c.p, c.y); }
        else if constexpr (MN == TXA) { c.a = c.x; c.p = nz(c.p, c.a); }
        else if constexpr (MN == TYA) { c.a = c.y; c.p = nz(c.p, c.a); }
        else if constexpr (MN == TSX) { c.x = c.sp; c.p = nz(c.p, c.x); }
        else if constexpr (MN == TXS) { c.sp = c.x; }
        else if constexpr (MN == CLC) { c.p &= ~FC; }
        else if constexpr (MN == SEC) { c.p |= FC; }
        else if constexpr (MN == CLI) { c.p &= ~FI; }
        else if constexpr (MN == SEI) { c.p |= FI; }
        else if constexpr (MN == CLV) { c.p &= ~FV; }
        else if constexpr (MN == CLD) { c.p &= ~FD; }
        else if constexpr (MN == SED) { c.p |= FD; }
        F.pc = next;
        F.cyc += N;
        return FS_NEXT;
    } else if constexpr (MD == ZP || MD == ABS) {
        const uint32_t ea = MD == ZP ? b1 : (b1 | (b2 << 8));
        const uint32_t a = ea & 0x1FFF;
        const uint32_t t = F.cyc + N - 1;
        if constexpr (MN == JMP) {
            F.pc = ea;
            F.cyc += N;
            return FS_NEXT;
        } else if constexpr (MN == JSR) {
            if (!all_lanes(c.sp >= 0x81)) return FS_EXIT;
            const uint32_t ret = (next - 1) & 0xFFFF;
            W.ram[c.ram_off + (c.sp & 0x7F)] = (uint8_t)(ret >> 8);
            W.ram[c.ram_off + ((c.sp - 1) & 0x7F)] = (uint8_t)(ret & 0xFF);
            c.sp = (c.sp - 2) & 0xFF;
            F.pc = ea;
            F.cyc += N;
            return FS_NEXT;
        } else if constexpr (read_mn(MN)) {
            uint32_t dm = 0;
            if constexpr (MN == ADC || MN == SBC) {
                dm = dec_mode(c);
                if (dm == 2) return FS_EXIT;
            }
            uint32_t v;
            if constexpr (HOT && MD == ZP) {
                // unmarked zero-page read: RAM (reads below $80 are marked)
                v = W.ram[c.ram_off + (a & 0x7F)];
            } else {
                if (TRACK && aux == SC_EXIT) return FS_EXIT;   // a latch read: the per-lane path scans the log
                if (MD == ABS && aux == SC_XRAM)      // Superchip RAM: read port, or the write port (0)
                    v = (a & 0x80) ? (uint32_t)c.xram[a & 0x7F] : 0u;
                else
                    v = fast_rd(c, W, F, a, t);
            }
            fast_alu(c, MN, v, dm);
            F.pc = next;
            F.cyc += N;
            return FS_NEXT;
        } else if constexpr (store_mn(MN)) {
            // aux is store_class(a), from the predecoded word
            const uint32_t v = store_value<MN>(c);
            if (aux == SC_RAM) {
                W.ram[c.ram_off + (a & 0x7F)] = (uint8_t)v;
            } else if (aux >= SC_TIA) {
                // from the hot loop a zero-page store is not an object reset or enable (marked)
                if (!fast_tia_code<(HOT && MD == ZP) ? 2 : 0>(c, W, F, aux, v & 0xFF, t)) return FS_EXIT;
            } else if (aux == SC_WSYNC) {
                return fast_finish(F, next, t, 1);
            } else if (aux == SC_EXIT) {
                return FS_EXIT;
            } else if (aux == SC_CART) {
                F.bank = hotspot(W, F.bank, a);
            } else if (aux == SC_XRAM) {
                if (!(a & 0x80)) c.xram[a & 0x7F] = (uint8_t)v;   // writes to the read port do nothing
            } else if (aux == SC_3F) {
                // the slice number must agree across the lanes to stay uniform
                const uint32_t sl = v & cm_tf_mask(W), s0 = rfl(sl);
                if (!all_lanes(sl == s0)) return FS_EXIT;
                F.bank = s0;
            }
            F.pc = next;
            F.cyc += N;
            return FS_NEXT;
        } else {
            static_assert(rmw_mn(MN), "read-modify-write");
            // a TIA register reads back as an input port or 0: RMW on one is
            // left to the per-lane path, as are the stores fast_store_ok refuses
            if (!(a & 0x1000) && !(a & 0x80)) return FS_EXIT;
            if (!fast_store_ok(a)) return FS_EXIT;
            if constexpr (MD == ABS) {
                if (aux == SC_XRAM) return FS_EXIT;   // RMW on the Superchip RAM window
            }
            const uint32_t v = fast_rd(c, W, F, a, t);
            const uint32_t r = fast_rmw(c, MN, v);
            uint32_t wsync = 0;
            fast_wr(c, W, F, a, r, t, wsync);
            return fast_finish(F, next, t, wsync);
        }
    } else if constexpr (MD == ZPX || MD == ZPY || MD == ABX || MD == ABY) {
        const uint32_t idx = (MD == ZPX || MD == ABX) ? c.x : c.y;
        uint32_t ea;
        bool cross = false;
        if constexpr (MD == ZPX || MD == ZPY) {
            ea = (b1 + idx) & 0xFF;
        } else {
            const uint32_t base = b1 | (b2 << 8);
            ea = (base + idx) & 0xFFFF;
            cross = ((base ^ ea) & 0xFF00) != 0;
        }
        const uint32_t a = ea & 0x1FFF;
        const bool in_ram = (a & 0x1280) == 0x0080;
        if constexpr (read_mn(MN)) {
            // cartridge addresses that are plain ROM: no hotspot, no Superchip RAM
            const bool in_cart = (a & 0x1000) && hotspot(W, F.bank, a) == F.bank && !sc_window(W, a);
            if (!all_lanes(in_ram || in_cart)) return FS_EXIT;
        } else {
            if (!all_lanes(in_ram)) return FS_EXIT;
        }
        uint32_t n = N;
        if constexpr (I.pen) {
            const uint32_t cr = rfl(cross ? 1u : 0u);
            if (!all_lanes(cross == (cr != 0))) return FS_EXIT;
            n += cr;
        }
        if constexpr (read_mn(MN)) {
            uint32_t dm = 0;
            if constexpr (MN == ADC || MN == SBC) {
                dm = dec_mode(c);
                if (dm == 2) return FS_EXIT;
            }
            // one LDS read from RAM or cartridge, whichever each lane's address is in
            const uint8_t* src = in_ram ? W.ram + c.ram_off + (a & 0x7F) : W.rom + rom_off(W, F.bank, a);
            fast_alu(c, MN, *src, dm);
        } else if constexpr (store_mn(MN)) {
            W.ram[c.ram_off + (a & 0x7F)] = (uint8_t)store_value<MN>(c);
        } else {
            static_assert(rmw_mn(MN), "read-modify-write");
            uint8_t* m = &W.ram[c.ram_off + (a & 0x7F)];
            *m = (uint8_t)fast_rmw(c, MN, *m);
        }
        F.pc = next;
        F.cyc += n;
        return FS_NEXT;
    } else {
        static_assert(MD == REL, "branch");
        bool taken;
        if constexpr (MN == BPL) taken = !(c.p & FN);
        else if constexpr (MN == BMI) taken = (c.p & FN) != 0;
        else if constexpr (MN == BVC) taken = !(c.p & FV);
        else if constexpr (MN == BVS) taken = (c.p & FV) != 0;
        else if constexpr (MN == BCC) taken = !(c.p & FC);
        else if constexpr (MN == BCS) taken = (c.p & FC) != 0;
        else if constexpr (MN == BNE) taken = !(c.p & FZ);
        else taken = (c.p & FZ) != 0;
        const uint32_t tgt = (next + (uint32_t)sext8(b1)) & kPcMask;
        const uint32_t extra = 1 + (((tgt ^ next) & 0xFF00) ? 1 : 0);
        const uint64_t tk = __builtin_amdgcn_ballot_w64(taken);
        if (tk == 0) {
            F.pc = next;
            F.cyc += N;
            return FS_NEXT;
        }
        if (tk == __builtin_amdgcn_ballot_w64(true)) {
            F.pc = tgt;
            F.cyc += N + extra;
            return FS_NEXT;
        }
        c.pc = taken ? tgt : next;            // the lanes part here
        c.cyc = F.cyc + N + (taken ? extra : 0);
        return FS_LANE;
    }
}

#define VCS_FAST_CASE(o) \
    case (o): st = fop<(o), TRACK>(c, W, F, b1, b2, aux); break;
#define VCS_FAST_4(o) VCS_FAST_CASE(o) VCS_FAST_CASE((o) + 1) VCS_FAST_CASE((o) + 2) VCS_FAST_CASE((o) + 3)
#define VCS_FAST_16(o) VCS_FAST_4(o) VCS_FAST_4((o) + 4) VCS_FAST_4((o) + 8) VCS_FAST_4((o) + 12)
#define VCS_FAST_64(o) VCS_FAST_16(o) VCS_FAST_16((o) + 16) VCS_FAST_16((o) + 32) VCS_FAST_16((o) + 48)

// Runs instructions for the lanes in exec (which agree on the control
// state) until they part, a frame ends, or an instruction this path leaves
// to the per-lane path comes up; when other running lanes of the wave are
// elsewhere (`partial`), also at the first WSYNC, so that lanes that took
// different paths through a scanline meet again at the next line start.  On
// return `c` holds every lane's state; `ended`/`end_t` mark lanes whose frame
// ended.  Returns false when it made no progress (the per-lane path must then
// execute the instruction in the same iteration).
template <bool TRACK>
__device__ __forceinline__ bool run_fast(Cpu& c, const Wave& W, const uint32_t* pre, bool& ended, uint32_t& end_t,
                                         uint32_t partial) {
    Fast F;
    F.partial = partial;
    F.stop = 0;
    F.pc = rfl(c.pc);
    F.bank = rfl(c.bank);
    F.cyc = rfl(c.cyc);
    F.cap = rfl(c.cap);
    F.lim = F.cap;
    F.fl = rfl(c.fl);
    F.orow = (uint32_t)(rfl(c.open_row) + 1);
    F.ocnt = rfl(c.open_cnt);
    F.obase = rfl(c.open_base);
    F.logon = rfl(c.log != nullptr ? 1u : 0u);
    uint32_t done_n = 0;       // instructions executed on this path
    uint32_t st = FS_EXIT;
    uint32_t capped = 0;
    // Two loops: the inner one handles only the most frequent opcodes of
    // typical cartridge code, so few values merge at its back edge and the
    // compiler keeps the state in place; any other opcode goes through the
    // full dispatch once, then the inner loop resumes.  The pc is checked
    // against the cartridge window only on entry and after a full-dispatch
    // instruction: an instruction the inner loop runs is marked in the
    // predecoded word (bit 31) when it could leave the window (it ends
    // within 2 bytes of the bank's end, or is a branch whose target is
    // outside), and a marked word never matches a frequent opcode.  Zero-
    // page reads below $80 (TIA) are marked too, so the inner loop's reads
    // are RAM reads.
    for (;;) {
        uint32_t op = 0, b1 = 0, b2 = 0, aux = 0;
        uint32_t cold = 0;
        if (F.cyc >= F.lim) {
            capped = F.lim != 0;
            break;
        }
        if ((F.pc & 0x1FFF) - 0x1000u > 0xFFDu) {   // outside the cartridge, or too close to its end
            st = FS_EXIT;
            break;
        }
        for (;;) {
            if (F.cyc >= F.lim) {      // the frame's last cycle, or a stop
                capped = F.lim != 0;
                break;
            }
            const uint32_t q = pre[(F.bank << 12) | (F.pc & 0xFFF)];
            const uint32_t hq = q & 0x800000FFu;   // the opcode, or no frequent one when marked
            b1 = (q >> 8) & 0xFF;
            b2 = (q >> 16) & 0xFF;
            aux = (q >> 24) & 0x7F;
#define VCS_HOT(o)                                            \
    if (hq == (o)) {                                          \
        if ((st = fop<(o), TRACK, true>(c, W, F, b1, b2, aux)) != FS_NEXT) break; \
    }
            VCS_HOT(0x85)                    // STA zp
            else VCS_HOT(0xA5)               // LDA zp
            else VCS_HOT(0xD0)               // BNE
            else VCS_HOT(0xCA)               // DEX
            else VCS_HOT(0x25)               // AND zp
            else VCS_HOT(0x65)               // ADC zp
            else VCS_HOT(0x45)               // EOR zp
            else VCS_HOT(0xA9)               // LDA #
            else {
                op = q & 0xFF;
                cold = 1;
                break;
            }
#undef VCS_HOT
            ++done_n;
        }
        if (!cold) break;
        switch (op) {
            VCS_FAST_64(0x00)
            VCS_FAST_64(0x40)
            VCS_FAST_64(0x80)
            VCS_FAST_64(0xC0)
        }
        if (st != FS_NEXT) break;
        ++done_n;
    }
    if (capped) {
        c.err |= ERR_FRAME_CAP;
        ended = true;
        end_t = F.cyc - 1;
    }
    if (st == FS_LANE) ++done_n;
    if (st != FS_LANE) {                      // pc and cycle are still common to all lanes
        c.pc = F.pc;
        c.cyc = F.cyc;
    }
    c.icount += done_n;
    c.ucount += done_n;
    c.bank = F.bank;
    c.open_row = (int32_t)F.orow - 1;
    c.open_cnt = F.ocnt;
    c.open_base = F.obase;
    return done_n > 0 || capped;
}
#undef VCS_FAST_64
#undef VCS_FAST_16
#undef VCS_FAST_4
#undef VCS_FAST_CASE

// ------------------------------------------------- two-bank group runs
//
// On bank-switched cartridges, lanes can stand at the same address and cycle
// in two different banks.  Where the instruction there has the same opcode
// in both banks (operands may differ), the lanes still run it as one group:
// the predecoded words of both banks come from two scalar loads, dispatch,
// store class and timing stay scalar, and each lane takes its bank's
// operand bytes.  Covered: implied and accumulator instructions, immediates,
// zero-page reads of RAM, zero-page stores whose target class agrees (RAM,
// WSYNC, a TIA register stored as is, or one with no emulated effect),
// relative branches and absolute jumps (the lanes part where their targets
// differ), and absolute reads of the cartridge at one address in both banks
// (a bank hotspot among them: the run ends after it).  Anything else ends
// the run before executing it.

// One instruction with opcode OP; qa / qb: its predecoded word in bank A /
// bank B; in_b: the lane is in bank B.
template <int OP>
__device__ __forceinline__ uint32_t mop(Cpu& c, const Wave& W, Fast& F, bool in_b, uint32_t qa, uint32_t qb) {
    constexpr OpInfo I = decode(OP);
    constexpr int MD = I.md, MN = I.mn;
    constexpr uint32_t N = (uint32_t)I.cyc;
    const uint32_t next = (F.pc + (uint32_t)op_len(MD)) & 0xFFFF;
    const uint32_t a1 = (qa >> 8) & 0xFF, a2 = (qa >> 16) & 0xFF;   // bank A's operand bytes
    const uint32_t x1 = (qb >> 8) & 0xFF, x2 = (qb >> 16) & 0xFF;   // bank B's
    const uint32_t b1 = in_b ? x1 : a1;                              // the lane's
    if constexpr (MN == ILL || MN == BRK || MN == RTI || MN >= SLO || (MN == NOP && MD != IMP)) {
        return FS_EXIT;
    } else if constexpr (MD == IMP || MD == ACC) {
        return fop<OP, false>(c, W, F, 0, 0, 0);   // no operand bytes; memory only through the stack
    } else if constexpr (MD == IMM) {
        uint32_t dm = 0;
        if constexpr (MN == ADC || MN == SBC) {
            dm = dec_mode(c);
            if (dm == 2) return FS_EXIT;
        }
        fast_alu(c, MN, b1, dm);
        F.pc = next;
        F.cyc += N;
        return FS_NEXT;
    } else if constexpr (MD == ZP && read_mn(MN)) {
        if (!(a1 & x1 & 0x80)) return FS_EXIT;    // RAM in both banks' operands
        uint32_t dm = 0;
        if constexpr (MN == ADC || MN == SBC) {
            dm = dec_mode(c);
            if (dm == 2) return FS_EXIT;
        }
        fast_alu(c, MN, W.ram[c.ram_off + (b1 & 0x7F)], dm);
        F.pc = next;
        F.cyc += N;
        return FS_NEXT;
    } else if constexpr (MD == ZP && store_mn(MN)) {
        const uint32_t auxa = (qa >> 24) & 0x7F, auxb = (qb >> 24) & 0x7F;      // store classes
        const uint32_t cat = auxa < SC_TIA ? auxa : (auxa & 0xE0);
        if (cat != (auxb < SC_TIA ? auxb : (auxb & 0xE0))) return FS_EXIT;
        const uint32_t t = F.cyc + N - 1;
        const uint32_t v = store_value<MN>(c);
        if (cat == SC_RAM) {
            W.ram[c.ram_off + (b1 & 0x7F)] = (uint8_t)v;
        } else if (cat == SC_TIA) {
            if (!fast_tia_code<1>(c, W, F, in_b ? auxb : auxa, v & 0xFF, t)) return FS_EXIT;
        } else if (cat == SC_WSYNC) {
            return fast_finish(F, next, t, 1);
        } else if (cat != SC_IGNORE) {
            return FS_EXIT;
        }
        F.pc = next;
        F.cyc += N;
        return FS_NEXT;
    } else if constexpr (MD == REL) {
        bool taken;
        if constexpr (MN == BPL) taken = !(c.p & FN);
        else if constexpr (MN == BMI) taken = (c.p & FN) != 0;
        else if constexpr (MN == BVC) taken = !(c.p & FV);
        else if constexpr (MN == BVS) taken = (c.p & FV) != 0;
        else if constexpr (MN == BCC) taken = !(c.p & FC);
        else if constexpr (MN == BCS) taken = (c.p & FC) != 0;
        else if constexpr (MN == BNE) taken = !(c.p & FZ);
        else taken = (c.p & FZ) != 0;
        const uint32_t tgt = (next + (uint32_t)sext8(b1)) & 0xFFFF;
        const uint32_t npc = taken ? tgt : next;
        const uint32_t ncyc = F.cyc + N + (taken ? 1 + (((tgt ^ next) & 0xFF00) ? 1 : 0) : 0);
        const uint32_t p0 = rfl(npc), c0 = rfl(ncyc);
        if (all_lanes(npc == p0 && ncyc == c0)) {
            F.pc = p0;
            F.cyc = c0;
            return FS_NEXT;
        }
        c.pc = npc;                           // the lanes part here
        c.cyc = ncyc;
        return FS_LANE;
    } else if constexpr (MN == JMP && MD == ABS) {
        const uint32_t ta = a1 | (a2 << 8), tb = x1 | (x2 << 8);
        if (ta == tb) {
            F.pc = ta;
            F.cyc += N;
            return FS_NEXT;
        }
        c.pc = in_b ? tb : ta;
        c.cyc = F.cyc + N;
        return FS_LANE;
    } else if constexpr (MD == ABS && read_mn(MN)) {
        const uint32_t a = (a1 | (a2 << 8)) & 0x1FFF;
        if (a1 != x1 || a2 != x2 || !(a & 0x1000) || cm_sc(W)) return FS_EXIT;
        uint32_t dm = 0;
        if constexpr (MN == ADC || MN == SBC) {
            dm = dec_mode(c);
            if (dm == 2) return FS_EXIT;
        }
        // each lane reads its own bank, after the access's bank switch
        c.bank = hotspot(W, c.bank, a);
        fast_alu(c, MN, W.rom[rom_off(W, c.bank, a)], dm);
        F.pc = next;
        F.cyc += N;
        F.stop = 1;                           // the banks may have changed: regroup
        return FS_NEXT;
    } else {
        return FS_EXIT;
    }
}

#define VCS_MB_CASE(o) \
    case (o): st = mop<(o)>(c, W, F, in_b, qa, qb); break;
#define VCS_MB_4(o) VCS_MB_CASE(o) VCS_MB_CASE((o) + 1) VCS_MB_CASE((o) + 2) VCS_MB_CASE((o) + 3)
#define VCS_MB_16(o) VCS_MB_4(o) VCS_MB_4((o) + 4) VCS_MB_4((o) + 8) VCS_MB_4((o) + 12)
#define VCS_MB_64(o) VCS_MB_16(o) VCS_MB_16((o) + 16) VCS_MB_16((o) + 32) VCS_MB_16((o) + 48)

// Runs the lanes in exec (same address, cycle, frame line and row-log
// position; each in bank `ba` or `bb` of a linearly mapped cartridge, both
// present) while the opcode agrees and mop covers it.  Same contract as
// run_fast; `in_b`: the lane is in bank bb.
__device__ __forceinline__ bool run_mb(Cpu& c, const Wave& W, const uint32_t* pre, bool& ended, uint32_t& end_t,
                                       uint32_t partial, uint32_t ba, uint32_t bb, bool in_b) {
    Fast F;
    F.partial = partial;
    F.stop = 0;
    F.pc = rfl(c.pc);
    F.bank = ba;
    F.cyc = rfl(c.cyc);
    F.cap = rfl(c.cap);
    F.lim = F.cap;
    F.fl = rfl(c.fl);
    F.orow = (uint32_t)(rfl(c.open_row) + 1);
    F.ocnt = rfl(c.open_cnt);
    F.obase = rfl(c.open_base);
    F.logon = rfl(c.log != nullptr ? 1u : 0u);
    uint32_t done_n = 0;
    uint32_t st = FS_EXIT;
    uint32_t capped = 0;
    for (;;) {
        if (F.cyc >= F.cap) {
            capped = 1;
            break;
        }
        if ((F.pc & 0x1FFF) - 0x1000u > 0xFFDu) {
            st = FS_EXIT;
            break;
        }
        const uint32_t qa = pre[(ba << 12) | (F.pc & 0xFFF)];
        const uint32_t qb = pre[(bb << 12) | (F.pc & 0xFFF)];
        const uint32_t op = qa & 0xFF;
        if ((qb & 0xFF) != op) {
            st = FS_EXIT;
            break;
        }
        switch (op) {
            VCS_MB_64(0x00)
            VCS_MB_64(0x40)
            VCS_MB_64(0x80)
            VCS_MB_64(0xC0)
        }
        if (st != FS_NEXT) break;
        ++done_n;
        if (F.stop) break;
    }
    if (capped) {
        c.err |= ERR_FRAME_CAP;
        ended = true;
        end_t = F.cyc - 1;
    }
    if (st == FS_LANE) ++done_n;
    if (st != FS_LANE) {
        c.pc = F.pc;
        c.cyc = F.cyc;
    }
    c.icount += done_n;
    c.ucount += done_n;
    c.open_row = (int32_t)F.orow - 1;
    c.open_cnt = F.ocnt;
    c.open_base = F.obase;
    return done_n > 0 || capped;
}
#undef VCS_MB_64
#undef VCS_MB_16
#undef VCS_MB_4
#undef VCS_MB_CASE

__device__ __forceinline__ uint32_t bcd_value(uint32_t b) { return 10 * (b >> 4) + (b & 15); }

// Minimum of v over the 64 lanes (call with every lane active): DPP swaps
// within quads, 8- and 16-lane mirrors, then row broadcasts; lane 63 ends up
// with the minimum.
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
    // the old value of a lane a step does not write is all ones (min's identity),
    // so each step folds into one DPP min
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x141, 0xF, 0xF, false));  // row_half_mirror
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x140, 0xF, 0xF, false));  // row_mirror
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x142, 0xA, 0xF, false));  // row_bcast:15
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)v, 0x143, 0xC, 0xF, false));  // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Lanes whose next instruction starts within this many cycles of the wave's
// earliest lane run together; the others wait.  Lanes of one ROM then meet
// again at every WSYNC line start and share one dispatch pass per instruction.
constexpr uint32_t kSchedWindow = 6;

// Next tile of a persistent launch (lane 0 takes it, the wave shares it).
__device__ __forceinline__ uint32_t take_tile(uint32_t* queue) {
    uint32_t t = 0;
    if (threadIdx.x == 0) t = atomicAdd(queue, 1u);
    return __builtin_amdgcn_readfirstlane(t);
}

// LL = envs a tile may hold (64 or 32): RAM and TIA registers get LL + 1
// slots in LDS (lanes at LL and above, always idle, share the last one), so
// narrow tiles take less LDS and more waves fit on a compute unit.
// RC = bytes of cartridge staged in LDS (8 KB), or 0: the cartridge is read
// from its HBM slot through the caches (launches with a ROM larger than 8 KB,
// which would otherwise need 32 KB of LDS per wave and cut the waves per CU
// by three).
// TRACK: collision latches tracked (the scan code exists only in that
// instantiation, so the other keeps its registers).  NOOPS: the reset no-op
// frames of restarted envs (envs with no frames to run leave at once, the
// step counter stays); a separate instantiation, so the step's kernel keeps
// its code.
template <int LL, int RC, bool TRACK, bool NOOPS>
__global__ void __launch_bounds__(kLanes) k_interp(InterpArgs A, const uint32_t* __restrict__ pre_all) {
    __shared__ uint32_t s_rom[RC ? RC / 4 + 4 : 1];
    __shared__ uint32_t s_ram[(LL + 1) * kRamStride / 4];
    __shared__ uint32_t s_tia[(LL + 1) * kTiaStride / 4];

    const uint32_t n_tiles = *A.n_tiles;
    uint32_t tile_id = A.queue ? take_tile(A.queue) : blockIdx.x;
    while (tile_id < n_tiles) {
        const Tile& T = A.tiles[tile_id];
        const int lane = threadIdx.x;
        const int rom_id = T.rom;

        Wave W;
        if constexpr (RC > 0) {   // stage the cartridge in LDS
            const uint4* rsrc = reinterpret_cast<const uint4*>(A.roms + (size_t)rom_id * kRomSlot);
            for (int i = lane; i < RC / 16; i += kLanes) reinterpret_cast<uint4*>(s_rom)[i] = rsrc[i];
            if (lane < 4) s_rom[RC / 4 + lane] = 0;
            W.rom = reinterpret_cast<const uint8_t*>(s_rom);
        } else {
            W.rom = A.roms + (size_t)rom_id * kRomSlot;
        }
        W.ram = reinterpret_cast<uint8_t*>(s_ram);
        W.tia = reinterpret_cast<uint8_t*>(s_tia);
        W.cm = A.cmap[rom_id];
        W.pre = pre_all + A.pre_off[rom_id];
        W.track = TRACK ? 1u : 0u;

        const int env = lane < T.count ? T.env[lane] : -1;
        const int out = lane < T.count ? T.out[lane] : 0;
        bool active = env >= 0;

        Cpu c;
        c.ram_off = (lane < LL ? lane : LL) * kRamStride;
        c.tia_off = (lane < LL ? lane : LL) * kTiaStride;
        c.ptr_memo = -1;
        DevEnv* E = active ? &A.envs[env] : nullptr;
        uint64_t base_line = 0;
        uint32_t prev_action = 0, act = 0, step_idx = 0, score0 = 0, nfr = A.nframes;
        uint64_t sticky_prefix = 0;
        if (active) {
            const uint4* src = reinterpret_cast<const uint4*>(E->ram);
            for (int i = 0; i < 8; ++i) {
                const uint4 q = src[i];
                uint32_t* d = s_ram + (c.ram_off >> 2) + 4 * i;
                d[0] = q.x; d[1] = q.y; d[2] = q.z; d[3] = q.w;
            }
            const uint4 qt = reinterpret_cast<const uint4*>(E->tia)[0];
            const uint4* q2 = reinterpret_cast<const uint4*>(E->tia2);
            uint32_t* dt = s_tia + (c.tia_off >> 2);
            dt[0] = qt.x; dt[1] = qt.y; dt[2] = qt.z; dt[3] = qt.w;
            for (int i = 0; i < 2; ++i) {
                const uint4 q = q2[i];
                dt[4 + 4 * i] = q.x; dt[5 + 4 * i] = q.y; dt[6 + 4 * i] = q.z; dt[7 + 4 * i] = q.w;
            }
            dt[12] = 0;
            c.a = E->a; c.x = E->x; c.y = E->y; c.sp = E->sp; c.p = E->p;
            c.bank = E->bank | ((uint32_t)E->bank_hi << 8);
            c.xram = E->xram;
            c.vsync = E->vsync; c.hmp0 = E->hmp0; c.hmp1 = E->hmp1;
            c.tv = E->tv; c.tshift = E->tshift; c.tbase = E->tbase;
            c.pc = E->pc;
            const uint64_t cyc = E->cycle;
            base_line = cyc / 76;
            c.cyc = (uint32_t)(cyc - base_line * 76);
            c.fl = (int32_t)((int64_t)E->frame_line0 - (int64_t)base_line);
            c.hmb_line = E->hmb_now ? 0 : -1;     // the line of `cycle` is the base line
            c.cx = E->cx;
            c.cx_need = -1;
            prev_action = E->prev_action;
            step_idx = E->step_idx;
            c.err = E->err;
            act = A.actions ? A.actions[out] : 0;
            if (A.nframes_per_out) nfr = A.nframes_per_out[out];
            sticky_prefix = rng_prefix(A.seed, (uint64_t)env, kStickyPurpose);
        }
        __syncthreads();
        score0 = active ? W.ram[c.ram_off + 0x50] : 0;
        c.base = base_line * 76;
        c.icount = 0;
        c.ucount = 0;
        c.slots = 0;
        c.slot = 0;
        c.log = nullptr;
        c.open_row = -1;
        c.open_cnt = 0;
        c.open_base = 0;
        c.tqm = 0;
        c.ev = 0;
        uint32_t k = 0, done = 0;
        uint32_t f = 0;
        uint32_t passes = 0;       // the wave's instruction passes (one per group instruction or opcode pass)
        uint32_t rounds = 0;       // its scheduling rounds (group formed, then scalar run or per-lane passes)

        auto begin_frame = [&]() {
            uint32_t eff = act;
            if (A.sticky_thr) {
                const uint64_t ctr = (uint64_t)step_idx * A.frameskip + f;
                if ((uint32_t)(rng_draw(sticky_prefix, ctr) >> 32) < A.sticky_thr) eff = prev_action;
            }
            prev_action = eff;
            c.swcha = (0xF0u & ~joy_pressed(eff)) | 0x0Fu;
            c.inpt4 = fire_pressed(eff) ? 0x00u : 0x80u;
            c.cap = 76u * (uint32_t)(320 + c.fl);
            const int32_t slot = A.render_all ? (int32_t)f : (int32_t)f - ((int32_t)nfr - 2);
            c.log = (A.log_enabled && slot >= 0 && slot < (int32_t)A.n_slots)
                        ? A.logs + ((size_t)out * A.n_slots + slot) * kFrameLogBytes
                        : nullptr;
            c.slot = (uint32_t)slot;
            c.log_scratch = 0;
            if (TRACK && !c.log) {                 // tracked collisions read every frame's log
                c.log = A.cx_logs + (size_t)out * kFrameLogBytes;
                c.log_scratch = 1;
            }
            c.open_row = -1;
            c.open_cnt = 0;
            c.open_base = 0;
            c.cx_row = 0;
            c.cx_x = 0;
            W.tia[c.tia_off + R_HMB] = 0;          // an earlier frame's blanked row is not this frame's
        };

        if constexpr (NOOPS) {
            if (nfr == 0) active = false;        // not restarted: nothing to run
        }
        if (active) {
            if (act >= 18) {
                c.err |= ERR_BAD_ACTION;
                done = 1;
                active = false;
            } else if (nfr == 0) {
                active = false;
            } else {
                begin_frame();
            }
        }

        // ---------------------------------------------------------- main loop
        while (__any(active)) {
            uint32_t op = 0, b1 = 0, b2 = 0;
            bool want = false, ended = false;
            uint32_t end_t = 0;
            // Scalar mode for the group of running lanes at exactly the place
            // of the earliest one (the whole wave when all lanes agree).
            bool uni = false;
            ++rounds;
            const uint32_t tmin = wave_min(active ? c.cyc : 0xFFFFFFFFu);
            const int lead = (int)__builtin_ctzll(__builtin_amdgcn_ballot_w64(active && c.cyc == tmin));
            uint32_t ran = 0;          // instructions the group ran on the scalar path
            if (active) {
                const uint32_t pc0 = rdl(c.pc, lead), bk0 = rdl(c.bank, lead);
                const int32_t fl0 = rdl(c.fl, lead), or0 = rdl(c.open_row, lead);
                const uint32_t oc0 = rdl(c.open_cnt, lead), ob0 = rdl(c.open_base, lead);
                const uint32_t lg0 = rdl(c.log != nullptr ? 1u : 0u, lead);
                const bool here = c.pc == pc0 && c.cyc == tmin && c.fl == fl0 && c.open_row == or0 &&
                                  c.open_cnt == oc0 && c.open_base == ob0 && (c.log != nullptr ? 1u : 0u) == lg0;
                const bool same = here && c.bank == bk0;
                bool mixed_ran = false;
                if constexpr (!TRACK && RC > 0) {
                    // lanes at the same place in a second bank: one group while the opcode agrees
                    // (launches with the cartridge staged in LDS: the 4 KB and 8 KB schemes; the
                    // instantiation for larger cartridges keeps its code without it)
                    const uint64_t other = __builtin_amdgcn_ballot_w64(here && !same);
                    if (cm_kind(W) == CART_LINEAR && other != 0) {
                        const uint32_t bb = rdl(c.bank, (int)__builtin_ctzll(other));
                        const bool grp = here && (c.bank == bk0 || c.bank == bb);
                        const uint32_t partial_grp = __builtin_amdgcn_ballot_w64(!grp) != 0 ? 1u : 0u;
                        if (grp) {
                            const uint32_t ic0 = c.icount;
                            uni = run_mb(c, W, W.pre, ended, end_t, partial_grp, bk0, bb, c.bank == bb);
                            ran = c.icount - ic0;
                        }
                        mixed_ran = __builtin_amdgcn_ballot_w64(uni) != 0;
                    }
                }
                if (!mixed_ran) {
                    const uint32_t partial = __builtin_amdgcn_ballot_w64(!same) != 0 ? 1u : 0u;
                    if (same) {
                        const uint32_t ic0 = c.icount;
                        uni = run_fast<TRACK>(c, W, W.pre, ended, end_t, partial);
                        ran = c.icount - ic0;
                    }
                }
            }
            passes += (uint32_t)__builtin_amdgcn_readlane((int)ran, lead);
            const bool ran_uniform = __any(uni);
            // A group ran and no lane's frame ended: nothing else happens this
            // round (no per-lane pass, no frame change), so the next round
            // starts at once; the short path back spares the common round
            // most of its bookkeeping.
            if (ran_uniform && !__any(ended)) continue;
            const bool go = !ran_uniform && active && c.cyc <= tmin + kSchedWindow;
            if (go) {
                if (c.cyc >= c.cap) {
                    c.err |= ERR_FRAME_CAP;
                    ended = true;
                    end_t = c.cyc - 1;
                } else {
                    const uint32_t pc = c.pc;
                    const uint32_t off = pc & 0xFFF;
                    if ((pc & 0x1000) && off <= 0xFFD) {
                        uint32_t v;
                        if (cm_kind(W) == CART_LINEAR) {   // the 4 KB bank is contiguous in LDS
                            const uint32_t boff = (c.bank << 12) | off;
                            const uint32_t* rw = reinterpret_cast<const uint32_t*>(W.rom);
                            const uint32_t w0 = rw[boff >> 2], w1 = rw[(boff >> 2) + 1];
                            v = __builtin_amdgcn_alignbyte(w1, w0, boff & 3);
                        } else {                          // segments: the predecoded word
                            v = W.pre[(c.bank << 12) | off];
                        }
                        op = v & 0xFF;
                        b1 = (v >> 8) & 0xFF;
                        b2 = (v >> 16) & 0xFF;
                    } else {
                        // bytes fetched from the TIA read registers show the
                        // latches through the fetch cycle's pixels, 3t+2
                        if constexpr (TRACK) cx_catch_up(c, W, 3 * (int32_t)c.cyc + 2);
                        op = peek(c, W, pc, c.cyc);
                        b1 = peek(c, W, pc + 1, c.cyc);
                        b2 = peek(c, W, pc + 2, c.cyc);
                    }
                    want = true;
                    c.ev = 0;
                    c.tqm = 0;
                }
            }
            // one pass per distinct opcode among the lanes that fetched one.
            // The instruction is counted, and `ran_lane` set, where it
            // completes: counting after the passes under the fetch mask
            // counted more instructions than ran in waves whose lanes took
            // the undocumented RRA / ISC at different places.
            bool todo = want;
            uint32_t ran_lane = 0;
            while (__any(todo)) {
                ++passes;
                if (todo) {
                    const uint32_t sop = __builtin_amdgcn_readfirstlane(op);
                    // an opaque scalar copy: inside the branch below the compiler
                    // would otherwise switch on the per-lane `op` (equal there)
                    uint32_t sw = sop;
                    asm volatile("" : "+s"(sw));
                    uint32_t d = kDecode.w[sw];
                    asm volatile("" : "+s"(d));
                    if (op == sop) {
                        if constexpr (TRACK) {
                            if (c.cx_need >= 0) {   // the second run of an instruction that read the latches
                                cx_catch_up(c, W, c.cx_need);
                                c.cx_need = -1;
                            }
                        }
                        const uint32_t sa = c.a, sx = c.x, sy = c.y, ssp = c.sp, sp_ = c.p, spc = c.pc,
                                       scy = c.cyc, sbk = c.bank;
                        exec_generic(d, c, W, b1, b2);
                        if (TRACK && c.cx_need >= 0) {   // undo; the latches are scanned before it runs again
                            c.a = sa; c.x = sx; c.y = sy; c.sp = ssp; c.p = sp_; c.pc = spc; c.cyc = scy;
                            c.bank = sbk;
                            c.tqm = 0;
                            c.ev = 0;
                        } else {
                            todo = false;
                            ran_lane = 1;
                            if (!(c.err & ERR_ILLEGAL)) c.icount++;
                            if constexpr (TRACK) c.ptr_memo = -1;
                        }
                    }
                }
            }
            if (ran_lane) {
                if (c.err & ERR_ILLEGAL) {
                    ended = true;
                    end_t = c.cyc - 1;
                } else {
                    const uint32_t t = c.ac;
                    apply_queue(c, W, t);
                    if (c.ev & EV_WSYNC) c.cyc = 76 * (t / 76 + 1);
                    if (c.ev & EV_VSYNC) {
                        ended = true;
                        end_t = t;
                    }
                }
            }
            // Every iteration moves some lane on (the earliest lane always
            // runs); if none moved, stop the wave's frames with an error
            // instead of spinning.
            if (!__any(ran_lane != 0 || uni || ended) && active) {
                c.err |= ERR_FRAME_CAP;
                ended = true;
                end_t = c.cyc;
            }
            if (ended) {
                if (c.log) {
                    uint8_t* lg = c.log;
                    log_close(c, W, end_t);
                    if constexpr (TRACK) {         // the latches take the frame's remaining rows
                        c.log = lg;
                        cx_catch_up(c, W, -1);
                        c.log = nullptr;
                    }
                }
                c.fl = (int32_t)(end_t / 76);
                ++k;
                ++f;
                const bool term = A.early_stop && W.ram[c.ram_off + 0x51] != 0;
                if (c.err || term) {
                    done = 1;
                    active = false;
                } else if (f >= nfr) {
                    active = false;
                } else {
                    begin_frame();
                }
            }
        }

        // ---------------------------------------------------------- write back
        if (env >= 0) {
            const uint32_t* sr = s_ram + (c.ram_off >> 2);
            uint4* dst = reinterpret_cast<uint4*>(E->ram);
            for (int i = 0; i < 8; ++i) dst[i] = make_uint4(sr[4 * i], sr[4 * i + 1], sr[4 * i + 2], sr[4 * i + 3]);
            const uint32_t* st = s_tia + (c.tia_off >> 2);
            reinterpret_cast<uint4*>(E->tia)[0] = make_uint4(st[0], st[1], st[2], st[3]);
            reinterpret_cast<uint4*>(E->tia2)[0] = make_uint4(st[4], st[5], st[6], st[7]);
            reinterpret_cast<uint4*>(E->tia2)[1] = make_uint4(st[8], st[9], st[10], st[11]);
            E->hmb_now = c.hmb_line >= 0 && (uint32_t)c.hmb_line == c.cyc / 76 ? 1 : 0;
            E->cx = (uint16_t)c.cx;
            E->a = c.a; E->x = c.x; E->y = c.y; E->sp = c.sp; E->p = c.p;
            E->bank = (uint8_t)c.bank;
            E->bank_hi = (uint8_t)(c.bank >> 8);
            E->vsync = c.vsync; E->hmp0 = c.hmp0; E->hmp1 = c.hmp1;
            E->tv = c.tv; E->tshift = c.tshift; E->tbase = c.tbase;
            E->pc = c.pc;
            E->cycle = c.base + c.cyc;
            E->frame_line0 = (uint64_t)((int64_t)base_line + c.fl);
            E->instr += c.icount;
            E->prev_action = prev_action;
            E->err = c.err;
            E->step_idx = step_idx + (NOOPS ? 0u : 1u);
            StepInfo si;
            si.k = (uint8_t)k;
            si.done = (uint8_t)done;
            si.err = (uint8_t)c.err;
            si.slots = (uint8_t)c.slots;
            A.info[out] = si;
            if (A.done) A.done[out] = (uint8_t)done;
            if (A.reward) {
                const uint32_t s1 = W.ram[c.ram_off + 0x50];
                A.reward[out] = (int32_t)bcd_value(s1) - (int32_t)bcd_value(score0);
            }
            if (c.err) {
                atomicOr(&A.err_word[0], c.err);
                atomicMin(&A.err_word[1], (uint32_t)env);
            }
            if (A.instr_total) {
                atomicAdd(&A.instr_total[0], (unsigned long long)c.icount);
                atomicAdd(&A.instr_total[1], (unsigned long long)c.ucount);
            }
        }
        if (A.instr_total && lane == 0) {
            atomicAdd(&A.instr_total[2], (unsigned long long)passes);
            atomicAdd(&A.instr_total[3], (unsigned long long)rounds);
        }
        if (!A.queue) break;
        __syncthreads();   // every lane is done with the LDS of this tile
        tile_id = take_tile(A.queue);
    }
}

// Predecoded ROM: for every virtual bank and offset, opcode | b1 << 8 |
// b2 << 16 | aux << 24 for the instruction that starts there (each byte read
// through the bank's mapping, so instructions that cross an E0 or 3F segment
// boundary decode exactly).  aux is the store class of the address of a
// zero-page or absolute STA/STX/STY; on 3F cartridges a store to $00-$3F
// (which also selects a slice) is SC_3F when the TIA register it reaches is
// not emulated, else SC_EXIT (left to the per-lane path); on Superchip
// cartridges an absolute access to the RAM window is SC_XRAM; with tracked
// collisions a zero-page / absolute read of a latch register is SC_EXIT
// (aux takes 7 bits).  Bit 31 marks an instruction the scalar hot loop
// leaves to the full dispatch: one after which the pc may leave the window
// $000-$FFD of the bank (it ends past $FFD, or is a branch whose target is
// outside), a zero-page read below $80 (a TIA read, not RAM), or a
// zero-page store to an object reset, enable or vertical-delay register.
// Entries past offset $FFD are never used.
__global__ void k_predecode(const uint8_t* rom, RomInfo R, uint32_t* pre, uint32_t track) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= R.n_vbanks * 4096u) return;
    const uint32_t bank = i >> 12, off = i & 0xFFF;
    const uint32_t op = rom[cart_rom_off(R, bank, 0x1000 | off)];
    const uint32_t b1 = off + 1 < 4096 ? rom[cart_rom_off(R, bank, 0x1000 | (off + 1))] : 0;
    const uint32_t b2 = off + 2 < 4096 ? rom[cart_rom_off(R, bank, 0x1000 | (off + 2))] : 0;
    const uint32_t d = kDecode.w[op];
    const uint32_t md = d & 15, abs_addr = (b1 | (b2 << 8)) & 0x1FFF;
    uint32_t aux = 0;
    const bool st = op == 0x84 || op == 0x85 || op == 0x86 || op == 0x8C || op == 0x8D || op == 0x8E;
    const uint32_t a = (op == 0x84 || op == 0x85 || op == 0x86) ? b1 : abs_addr;
    if (st) {
        aux = store_class(a);
        if (R.kind == CART_3F && a <= 0x3F) aux = aux == SC_IGNORE ? SC_3F : SC_EXIT;
    }
    if (R.sc && md == ABS && ((d >> DW_RD) & 1 || (d >> DW_WR) & 1) && (abs_addr & 0x1000) && !(abs_addr & 0xF00))
        aux = SC_XRAM;
    // tracked collision latches: zero-page / absolute reads of CXM0P..CXPPMM
    const uint32_t ra = md == ZP ? b1 : abs_addr;
    if (track && (md == ZP || md == ABS) && ((d >> DW_RD) & 1) && !((d >> DW_WR) & 1) && !(ra & 0x1080) && (ra & 0xF) < 8)
        aux = SC_EXIT;
    bool edge = off + ((d >> DW_LEN) & 3) > 0xFFD;
    if ((op & 0x1F) == 0x10) {             // conditional branch: its target
        const int32_t t = (int32_t)off + 2 + (int32_t)(int8_t)b1;
        edge = edge || t < 0 || t > 0xFFD;
    }
    if (md == ZP && ((d >> DW_RD) & 1) && b1 < 0x80) edge = true;   // a TIA read
    if (md == ZP && st && aux >= SC_TIAS && aux < SC_TIAG) edge = true;   // an object reset or enable
    pre[i] = op | (b1 << 8) | (b2 << 16) | (aux << 24) | ((edge ? 1u : 0u) << 31);
}

void launch_predecode(const uint8_t* rom, const RomInfo& info, uint32_t* pre, uint32_t track, hipStream_t s) {
    const uint32_t n = info.n_vbanks * 4096u;
    hipLaunchKernelGGL(k_predecode, dim3((n + 255) / 256), dim3(256), 0, s, rom, info, pre, track);
}

template <bool TRACK, bool NOOPS>
static void launch_interp_t(const InterpArgs& a, uint32_t grid, uint32_t tile_envs, uint32_t rom_lds, hipStream_t s) {
    if (rom_lds == 0) {
        if (tile_envs <= 32)
            hipLaunchKernelGGL((k_interp<32, 0, TRACK, NOOPS>), dim3(grid), dim3(kLanes), 0, s, a, a.pre);
        else
            hipLaunchKernelGGL((k_interp<64, 0, TRACK, NOOPS>), dim3(grid), dim3(kLanes), 0, s, a, a.pre);
    } else if (tile_envs <= 32) {
        hipLaunchKernelGGL((k_interp<32, 8192, TRACK, NOOPS>), dim3(grid), dim3(kLanes), 0, s, a, a.pre);
    } else {
        hipLaunchKernelGGL((k_interp<64, 8192, TRACK, NOOPS>), dim3(grid), dim3(kLanes), 0, s, a, a.pre);
    }
}

void launch_interp(const InterpArgs& a, uint32_t grid, uint32_t tile_envs, uint32_t rom_lds, hipStream_t s) {
    if (a.track) {
        if (a.count_step) launch_interp_t<true, false>(a, grid, tile_envs, rom_lds, s);
        else launch_interp_t<true, true>(a, grid, tile_envs, rom_lds, s);
    } else {
        if (a.count_step) launch_interp_t<false, false>(a, grid, tile_envs, rom_lds, s);
        else launch_interp_t<false, true>(a, grid, tile_envs, rom_lds, s);
    }
}

}  // namespace vcs
