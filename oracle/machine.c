/*
 * One Atari 2600 console, stepped cycle by cycle -- CPU oracle (test
 * infrastructure; see vcs_oracle.h).
 *
 * The paper (Section 3) names the parts -- the 6507 CPU, the 128 B RAM, the
 * cartridge ROM and the TIA that turns register writes into a 160x210 frame --
 * but gives none of their semantics.  This file writes them out from the public
 * hardware definition (MOS 6502 programming manual; Atari 2600 TIA and RIOT
 * register maps) with these conventions:
 *
 *  - Bus: 13 address lines.  a & $1000 -> cartridge; else a & $80 == 0 -> TIA
 *    (write register a & $3F, read register a & $0F); else a & $200 == 0 ->
 *    RAM[a & $7F]; else RIOT ports/timer.
 *  - Timing: an instruction that starts at cycle t and lasts n cycles makes
 *    all of its data accesses (operand, pointer, stack and vector reads and
 *    writes) at cycle t+n-1, in program order; opcode and operand bytes are
 *    fetched at cycle t without side effects.  Read-modify-write instructions
 *    write once.  Dummy reads are not performed.
 *  - Beam: cycle c shows colour clocks 3c, 3c+1, 3c+2 (228 clocks a line,
 *    76 cycles a line); a TIA write at cycle c affects clocks from 3(c+1) on.
 *  - WSYNC written at cycle c: the next instruction starts at 76*(c/76 + 1).
 *  - A frame ends after the instruction that writes VSYNC with bit 1 set while
 *    bit 1 was clear; frame row r is scanline 34 + r counted from the line of
 *    the write that began the frame, and column x is colour clock 68 + x.
 *    An instruction that would start 320 or more lines after the frame's first
 *    line ends the frame instead (FRAME_CAP); an undocumented opcode ends it
 *    too (ILLEGAL); both freeze the machine.
 *  - Power-on: A=X=Y=0, SP=$FD, P=$24, RAM and TIA zero, positions 0, timer
 *    interval 1024 with INTIM reading 0 from cycle 0 (phase 0), the last
 *    4 KB bank of F8/F6/F4 cartridges, E0 slices 4, 5, 6 in segments 0-2,
 *    3F slice 0, PC from the reset vector, cycle 0.
 *  - Cartridges (see the bank-switching section below): 2 or 4 KB flat;
 *    F8/F6/F4 with 2/4/8 banks of 4 KB picked by any data access to
 *    $FF8-$FF9 / $FF6-$FF9 / $FF4-$FFB (switch first, then the access);
 *    their Superchip forms with 128 B of extra RAM written at $1000-$107F and
 *    read at $1080-$10FF; E0 (8 x 1 KB slices, segment 3 fixed to slice 7,
 *    segment k of 0-2 set to slice n by an access to $FE0 + 8k + n); 3F
 *    (2 KB slices: the upper half fixed to the last one, the lower half set
 *    to slice v mod S by a write of v to $00-$3F, which also reaches the TIA).
 *  - TIA objects: players with NUSIZ copies (offsets 0/16/32/64 by mode) and
 *    double/quad width, missiles (ENAM, 1-8 pixels, the player's copies,
 *    hidden while RESMP is set and placed at the player's position + 3/6/10
 *    when it is released), the ball (ENABL, CTRLPF size), vertical delay (a
 *    GRP0 write copies GRP1 to its old register, a GRP1 write copies GRP0 and
 *    ENABL), RESM/RESBL at h < 68 ? 2 : h - 68 + 4, HMOVE moving all five by
 *    the extra motion pulses that fall in horizontal blank (the HM nibble's
 *    signed motion for a strobe early in the blank, less for later ones)
 *    and, when written before colour clock 68, blanking pixels 0-7 of its
 *    line; priority P0/M0 > P1/M1 > PF/BL > BK (PF/BL first with CTRLPF
 *    D2), the ball in COLUPF.
 *  - Collisions (when tracked): the 15 latches set at every drawn pixel of
 *    the 210 frame rows (VBLANK clear, outside an HMOVE blank) where two
 *    objects meet; a read at access cycle t sees pixels up to colour clock
 *    3t+2; CXCLR clears them; untracked, they read 0.  The TIA drives them
 *    on every read cycle of a collision register, so an opcode, operand or
 *    zero-page pointer byte fetched from one shows them too, through colour
 *    clock 3t+2 of the instruction's first cycle t.
 *  - Undocumented opcodes: the stable ones (SLO, RLA, SRE, RRA, SAX, LAX,
 *    DCP, ISC, ANC, ALR, ARR, SBX, LAS, SBC #, and the NOPs of every width,
 *    which perform their read) run with the operations, cycle counts and
 *    flags of the NMOS 6502's combined ALU/RMW behaviour; the twelve JAMs and
 *    the unstable ANE, LXA, SHA, SHX, SHY and TAS fault (ILLEGAL).
 */
#include "machine.h"

#include <string.h>

/* ------------------------------------------------------------------ decode */

enum {
    ADC, AND, ASL, BCC, BCS, BEQ, BIT, BMI, BNE, BPL, BRK, BVC, BVS, CLC, CLD, CLI, CLV,
    CMP, CPX, CPY, DEC, DEX, DEY, EOR, INC, INX, INY, JMP, JSR, LDA, LDX, LDY, LSR, NOP,
    ORA, PHA, PHP, PLA, PLP, ROL, ROR, RTI, RTS, SBC, SEC, SED, SEI, STA, STX, STY, TAX,
    TAY, TSX, TXA, TXS, TYA,
    SLO, RLA, SRE, RRA, SAX, LAX, DCP, ISC, ANC, ALR, ARR, SBX, LAS,
    ILL
};
enum { IMP, ACC, IMM, ZP, ZPX, ZPY, ABS, ABX, ABY, IZX, IZY, IND, REL };

typedef struct { uint8_t mn, mode; } Decoded;
static Decoded DEC_TABLE[256];
static int table_ready = 0;
static void build_table(void);
__attribute__((constructor)) static void init_table(void) { build_table(); }

static void def(int op, int mn, int mode) { DEC_TABLE[op].mn = (uint8_t)mn; DEC_TABLE[op].mode = (uint8_t)mode; }

/* The documented NMOS 6502 opcode matrix. */
static void build_table(void) {
    for (int i = 0; i < 256; i++) { DEC_TABLE[i].mn = ILL; DEC_TABLE[i].mode = IMP; }
    /* group of eight addressing modes shared by the ALU instructions */
    const int alu_mn[8] = {ORA, AND, EOR, ADC, -1, LDA, CMP, SBC};
    for (int g = 0; g < 8; g++) {
        if (alu_mn[g] < 0) continue;
        int base = g << 5;
        def(base | 0x01, alu_mn[g], IZX);
        def(base | 0x05, alu_mn[g], ZP);
        def(base | 0x09, alu_mn[g], IMM);
        def(base | 0x0D, alu_mn[g], ABS);
        def(base | 0x11, alu_mn[g], IZY);
        def(base | 0x15, alu_mn[g], ZPX);
        def(base | 0x19, alu_mn[g], ABY);
        def(base | 0x1D, alu_mn[g], ABX);
    }
    /* STA: the same pattern without immediate */
    def(0x81, STA, IZX); def(0x85, STA, ZP); def(0x8D, STA, ABS); def(0x91, STA, IZY);
    def(0x95, STA, ZPX); def(0x99, STA, ABY); def(0x9D, STA, ABX);
    /* shifts, rotates, INC, DEC */
    const int sh_mn[4] = {ASL, ROL, LSR, ROR};
    for (int g = 0; g < 4; g++) {
        int base = g << 5;
        def(base | 0x06, sh_mn[g], ZP);
        def(base | 0x0A, sh_mn[g], ACC);
        def(base | 0x0E, sh_mn[g], ABS);
        def(base | 0x16, sh_mn[g], ZPX);
        def(base | 0x1E, sh_mn[g], ABX);
    }
    def(0xC6, DEC, ZP); def(0xCE, DEC, ABS); def(0xD6, DEC, ZPX); def(0xDE, DEC, ABX);
    def(0xE6, INC, ZP); def(0xEE, INC, ABS); def(0xF6, INC, ZPX); def(0xFE, INC, ABX);
    /* loads and stores of X and Y */
    def(0xA2, LDX, IMM); def(0xA6, LDX, ZP); def(0xAE, LDX, ABS); def(0xB6, LDX, ZPY); def(0xBE, LDX, ABY);
    def(0xA0, LDY, IMM); def(0xA4, LDY, ZP); def(0xAC, LDY, ABS); def(0xB4, LDY, ZPX); def(0xBC, LDY, ABX);
    def(0x86, STX, ZP); def(0x8E, STX, ABS); def(0x96, STX, ZPY);
    def(0x84, STY, ZP); def(0x8C, STY, ABS); def(0x94, STY, ZPX);
    /* compares with X and Y, BIT */
    def(0xE0, CPX, IMM); def(0xE4, CPX, ZP); def(0xEC, CPX, ABS);
    def(0xC0, CPY, IMM); def(0xC4, CPY, ZP); def(0xCC, CPY, ABS);
    def(0x24, BIT, ZP); def(0x2C, BIT, ABS);
    /* branches */
    def(0x10, BPL, REL); def(0x30, BMI, REL); def(0x50, BVC, REL); def(0x70, BVS, REL);
    def(0x90, BCC, REL); def(0xB0, BCS, REL); def(0xD0, BNE, REL); def(0xF0, BEQ, REL);
    /* jumps, subroutines, interrupts */
    def(0x4C, JMP, ABS); def(0x6C, JMP, IND); def(0x20, JSR, ABS);
    def(0x60, RTS, IMP); def(0x40, RTI, IMP); def(0x00, BRK, IMP);
    /* stack */
    def(0x48, PHA, IMP); def(0x08, PHP, IMP); def(0x68, PLA, IMP); def(0x28, PLP, IMP);
    /* flags */
    def(0x18, CLC, IMP); def(0x38, SEC, IMP); def(0x58, CLI, IMP); def(0x78, SEI, IMP);
    def(0xB8, CLV, IMP); def(0xD8, CLD, IMP); def(0xF8, SED, IMP);
    /* register transfers and increments */
    def(0xAA, TAX, IMP); def(0xA8, TAY, IMP); def(0xBA, TSX, IMP); def(0x8A, TXA, IMP);
    def(0x9A, TXS, IMP); def(0x98, TYA, IMP);
    def(0xCA, DEX, IMP); def(0x88, DEY, IMP); def(0xE8, INX, IMP); def(0xC8, INY, IMP);
    def(0xEA, NOP, IMP);

    /* undocumented, stable: the read-modify-write + ALU pairs share the
       eight-mode pattern of the ALU group (cc = 3) */
    const int combo_mn[8] = {SLO, RLA, SRE, RRA, -1, -1, DCP, ISC};
    for (int g = 0; g < 8; g++) {
        if (combo_mn[g] < 0) continue;
        int base = (g << 5) | 3;
        def(base | 0x00, combo_mn[g], IZX);
        def(base | 0x04, combo_mn[g], ZP);
        def(base | 0x0C, combo_mn[g], ABS);
        def(base | 0x10, combo_mn[g], IZY);
        def(base | 0x14, combo_mn[g], ZPX);
        def(base | 0x18, combo_mn[g], ABY);
        def(base | 0x1C, combo_mn[g], ABX);
    }
    def(0x83, SAX, IZX); def(0x87, SAX, ZP); def(0x8F, SAX, ABS); def(0x97, SAX, ZPY);
    def(0xA3, LAX, IZX); def(0xA7, LAX, ZP); def(0xAF, LAX, ABS); def(0xB3, LAX, IZY);
    def(0xB7, LAX, ZPY); def(0xBF, LAX, ABY);
    def(0xBB, LAS, ABY);
    def(0x0B, ANC, IMM); def(0x2B, ANC, IMM); def(0x4B, ALR, IMM); def(0x6B, ARR, IMM);
    def(0xCB, SBX, IMM); def(0xEB, SBC, IMM);
    /* NOPs: implied, immediate, zero page, zero page,X, absolute, absolute,X */
    const int nop_imp[6] = {0x1A, 0x3A, 0x5A, 0x7A, 0xDA, 0xFA};
    const int nop_imm[5] = {0x80, 0x82, 0x89, 0xC2, 0xE2};
    const int nop_zp[3] = {0x04, 0x44, 0x64};
    const int nop_zpx[6] = {0x14, 0x34, 0x54, 0x74, 0xD4, 0xF4};
    const int nop_abx[6] = {0x1C, 0x3C, 0x5C, 0x7C, 0xDC, 0xFC};
    for (int i = 0; i < 6; i++) { def(nop_imp[i], NOP, IMP); def(nop_zpx[i], NOP, ZPX); def(nop_abx[i], NOP, ABX); }
    for (int i = 0; i < 5; i++) def(nop_imm[i], NOP, IMM);
    for (int i = 0; i < 3; i++) def(nop_zp[i], NOP, ZP);
    def(0x0C, NOP, ABS);
    table_ready = 1;
}

static int is_store(int mn) { return mn == STA || mn == STX || mn == STY || mn == SAX; }
static int is_rmw(int mn) { return mn == ASL || mn == LSR || mn == ROL || mn == ROR || mn == INC || mn == DEC; }
/* undocumented read-modify-write + ALU pairs */
static int is_combo(int mn) {
    return mn == SLO || mn == RLA || mn == SRE || mn == RRA || mn == DCP || mn == ISC;
}

/* Base cycle count of an instruction (MOS programming manual, Appendix A). */
static int base_cycles(int mn, int mode) {
    switch (mn) {
    case BRK: return 7;
    case JSR: case RTS: case RTI: return 6;
    case PHA: case PHP: return 3;
    case PLA: case PLP: return 4;
    case JMP: return mode == IND ? 5 : 3;
    default: break;
    }
    if (mode == REL) return 2;
    if (mode == IMP) return 2;
    if (is_combo(mn)) {
        switch (mode) {
        case ZP: return 5; case ZPX: return 6; case ABS: return 6; case ABX: case ABY: return 7;
        case IZX: case IZY: return 8;
        }
    }
    if (is_rmw(mn)) {
        switch (mode) {
        case ACC: return 2; case ZP: return 5; case ZPX: return 6; case ABS: return 6; case ABX: return 7;
        }
    }
    if (is_store(mn)) {
        switch (mode) {
        case ZP: return 3; case ZPX: case ZPY: return 4; case ABS: return 4;
        case ABX: case ABY: return 5; case IZX: return 6; case IZY: return 6;
        }
    }
    switch (mode) {   /* read instructions */
    case IMM: return 2; case ZP: return 3; case ZPX: case ZPY: return 4; case ABS: return 4;
    case ABX: case ABY: return 4; case IZX: return 6; case IZY: return 5;
    }
    return 2;
}

/* ---------------------------------------------------------------- devices */

/* ------------------------------------------------------- bank switching */

static int linear_banks(uint32_t scheme) {
    switch (scheme) {
    case SCH_F8: case SCH_F8SC: return 2;
    case SCH_F6: case SCH_F6SC: return 4;
    case SCH_F4: case SCH_F4SC: return 8;
    default: return 1;
    }
}
static int has_superchip(uint32_t scheme) {
    return scheme == SCH_F8SC || scheme == SCH_F6SC || scheme == SCH_F4SC;
}

/* ROM sizes each scheme takes */
int m_rom_size_ok(uint32_t size, uint32_t scheme) {
    switch (scheme) {
    case SCH_4K: return size == 2048 || size == 4096;
    case SCH_E0: return size == 8192;
    case SCH_3F: return size == 4096 || size == 8192 || size == 16384 || size == 32768;
    default: return scheme < SCH_COUNT && size == 4096u * (uint32_t)linear_banks(scheme);
    }
}

/* the ROM byte that cartridge address a (A12 set) shows under the current bank state */
static uint8_t rom_byte(const OMachine* m, uint16_t a) {
    uint32_t lo = a & 0xFFF;
    uint32_t off;
    if (m->scheme == SCH_E0) {
        uint32_t seg = lo >> 10;
        uint32_t slice = seg == 3 ? 7 : (m->bank >> (3 * seg)) & 7;
        off = slice * 1024 + (lo & 0x3FF);
    } else if (m->scheme == SCH_3F) {
        off = lo < 0x800 ? (uint32_t)m->bank * 2048 + lo : m->rom_size - 2048 + (lo - 0x800);
    } else if (m->scheme == SCH_4K) {
        off = lo % m->rom_size;                      /* a 2 KB ROM shows twice */
    } else {
        off = (uint32_t)m->bank * 4096 + lo;
    }
    return m->rom[off];
}

/* Hotspots of a data access to cartridge address a (before the access). */
static void cart_access(OMachine* m, uint16_t a) {
    uint32_t lo = a & 0xFFF;
    int nb = linear_banks(m->scheme);
    if (nb > 1) {
        uint32_t first = nb == 2 ? 0xFF8 : (nb == 4 ? 0xFF6 : 0xFF4);
        if (lo >= first && lo < first + (uint32_t)nb) m->bank = (uint16_t)(lo - first);
    } else if (m->scheme == SCH_E0 && lo >= 0xFE0 && lo <= 0xFF7) {
        uint32_t seg = (lo - 0xFE0) / 8, slice = lo & 7;
        m->bank = (uint16_t)((m->bank & ~(7u << (3 * seg))) | (slice << (3 * seg)));
    }
}

/* data read of cartridge address a: hotspots, the Superchip RAM window, ROM */
static uint8_t cart_read(OMachine* m, uint16_t a) {
    cart_access(m, a);
    uint32_t lo = a & 0xFFF;
    if (has_superchip(m->scheme) && lo < 0x100)
        return lo < 0x80 ? 0x00 : m->xram[lo & 0x7F];   /* the write port reads as 0 */
    return rom_byte(m, a);
}

static void cart_write(OMachine* m, uint16_t a, uint8_t v) {
    cart_access(m, a);
    uint32_t lo = a & 0xFFF;
    if (has_superchip(m->scheme) && lo < 0x80) m->xram[lo] = v;   /* writes to the read port do nothing */
}

/* TIA read register reg, with the collision latches `cx` the read sees */
static uint8_t tia_read_with(const OMachine* m, uint16_t reg, uint16_t cx) {
    if ((reg & 0x0F) < 8)              /* CXM0P .. CXPPMM: latches in D7, D6 */
        return m->track_cx ? (uint8_t)(((cx >> (2 * (reg & 7))) & 3) << 6) : 0;
    switch (reg & 0x0F) {
    case 0x0C: return m->inpt4;        /* INPT4: fire button of player 0 */
    case 0x0D: return 0x80;            /* INPT5: player 1 button never pressed */
    default: return 0x00;              /* paddles, undriven bits */
    }
}

/* a data read at the access cycle: the beam has drawn that cycle's clocks */
static uint8_t tia_read(const OMachine* m, uint16_t reg) { return tia_read_with(m, reg, m->cx); }

static uint8_t riot_read(const OMachine* m, uint16_t a) {
    if ((a & 0x04) == 0) {
        switch (a & 3) {
        case 0: return m->swcha;
        case 2: return 0x0B;           /* SWCHB: no reset/select, colour, B difficulty */
        default: return 0x00;          /* data direction registers */
        }
    }
    if ((a & 1) == 0) return m->tim_count;            /* INTIM */
    return m->tim_expired ? 0x80 : 0x00;              /* TIMINT */
}

static void riot_write(OMachine* m, uint16_t a, uint8_t v) {
    static const uint16_t interval[4] = {1, 8, 64, 1024};
    if ((a & 0x14) != 0x14) return;    /* only the timer writes are honoured */
    m->tim_count = v;
    m->tim_sub = 0;
    m->tim_interval = interval[a & 3];
    m->tim_expired = 0;
    m->timer_written = 1;              /* this is the state as of the next cycle */
}

/* One cycle of the RIOT interval timer. */
static void timer_cycle(OMachine* m) {
    if (m->tim_expired) { m->tim_count = (uint8_t)(m->tim_count - 1); return; }
    m->tim_sub++;
    if (m->tim_sub == m->tim_interval) {
        m->tim_sub = 0;
        if (m->tim_count == 0) { m->tim_expired = 1; m->tim_count = 0xFF; }
        else m->tim_count--;
    }
}

static void tia_write(OMachine* m, uint16_t reg, uint8_t v) {
    uint32_t h_eff = (uint32_t)((3 * (m->access_cycle + 1)) % 228);
    switch (reg & 0x3F) {
    case 0x00:
        if ((v & 2) && !(m->vsync & 2)) m->vsync_on = 1;
        m->vsync = v; break;
    case 0x01: m->vblank = v; break;
    case 0x02: m->wsync_hit = 1; break;
    case 0x06: m->colup0 = v; break;
    case 0x07: m->colup1 = v; break;
    case 0x08: m->colupf = v; break;
    case 0x09: m->colubk = v; break;
    case 0x0A: m->ctrlpf = v; break;
    case 0x0B: m->refp0 = v; break;
    case 0x0C: m->refp1 = v; break;
    case 0x0D: m->pf0 = v; break;
    case 0x0E: m->pf1 = v; break;
    case 0x0F: m->pf2 = v; break;
    case 0x10: m->p0x = (uint8_t)(h_eff < 68 ? 3 : (h_eff - 68 + 5) % 160); break;
    case 0x11: m->p1x = (uint8_t)(h_eff < 68 ? 3 : (h_eff - 68 + 5) % 160); break;
    case 0x12: m->m0x = (uint8_t)(h_eff < 68 ? 2 : (h_eff - 68 + 4) % 160); break;
    case 0x13: m->m1x = (uint8_t)(h_eff < 68 ? 2 : (h_eff - 68 + 4) % 160); break;
    case 0x14: m->blx = (uint8_t)(h_eff < 68 ? 2 : (h_eff - 68 + 4) % 160); break;
    case 0x04: m->nusiz0 = v; break;
    case 0x05: m->nusiz1 = v; break;
    case 0x1B: m->grp0 = v; m->grp1_old = m->grp1; break;
    case 0x1C: m->grp1 = v; m->grp0_old = m->grp0; m->enabl_old = m->enabl; break;
    case 0x1D: m->enam0 = v; break;
    case 0x1E: m->enam1 = v; break;
    case 0x1F: m->enabl = v; break;
    case 0x20: m->hmp0 = v; break;
    case 0x21: m->hmp1 = v; break;
    case 0x22: m->hmm0 = v; break;
    case 0x23: m->hmm1 = v; break;
    case 0x24: m->hmbl = v; break;
    case 0x25: m->vdelp0 = v; break;
    case 0x26: m->vdelp1 = v; break;
    case 0x27: m->vdelbl = v; break;
    case 0x28: case 0x29: {            /* RESMP: release puts the missile at the player's centre */
        static const uint8_t CENTRE[8] = {3, 3, 3, 3, 3, 6, 3, 10};
        if (reg == 0x28) {
            if (!(v & 2) && (m->resmp0 & 2)) m->m0x = (uint8_t)((m->p0x + CENTRE[m->nusiz0 & 7]) % 160);
            m->resmp0 = v;
        } else {
            if (!(v & 2) && (m->resmp1 & 2)) m->m1x = (uint8_t)((m->p1x + CENTRE[m->nusiz1 & 7]) % 160);
            m->resmp1 = v;
        }
        break;
    }
    case 0x2A: {
        /* HMOVE.  After the strobe at clock h the TIA sends up to 15 extra
           motion pulses, one every 4 clocks (clocks h+4, h+8, ..., the
           count running on into the next line); an object takes its first
           n = (HM nibble) XOR 8 of them, and a pulse moves it one pixel left
           only where its position counter is not clocked anyway: in
           horizontal blank (clocks 0-67 of a line, 0-75 on a line whose
           blank the strobe extended).  A strobe before clock 68 extends its
           line's blank by 8 clocks, which withholds 8 ordinary clocks (8
           pixels right).  The strobe early in the blank gives the nibble's
           signed motion; late strobes lose the pulses that fall in the
           visible part.  The resulting move is applied now. */
        const uint8_t hm[5] = {m->hmp0, m->hmp1, m->hmm0, m->hmm1, m->hmbl};
        uint8_t* pos[5] = {&m->p0x, &m->p1x, &m->m0x, &m->m1x, &m->blx};
        const int extended = h_eff < 68;
        for (int i = 0; i < 5; i++) {
            const int n = ((hm[i] >> 4) & 0xF) ^ 8;
            int left = 0;
            for (int k = 1; k <= n; k++) {
                const uint32_t clk = h_eff + 4u * (uint32_t)k;   /* on the strobe's line, or past its end */
                const int blank = clk < 228 ? clk < (extended ? 76u : 68u) : clk - 228 < 68;
                if (blank) left++;
            }
            if (extended) left -= 8;
            *pos[i] = (uint8_t)(((int)*pos[i] - left + 320) % 160);
        }
        if (extended) m->hmove_blank_line = (int64_t)((m->access_cycle + 1) / 76);
        break;
    }
    case 0x2B: m->hmp0 = m->hmp1 = m->hmm0 = m->hmm1 = m->hmbl = 0; break;
    case 0x2C: m->cx = 0; break;
    default: break;                    /* audio and the rest: no emulated effect */
    }
}

/* data-access bus (side effects: bank switching, TIA and timer writes) */
static uint8_t bus_read(OMachine* m, uint16_t addr) {
    uint16_t a = addr & 0x1FFF;
    if (a & 0x1000) return cart_read(m, a);
    if ((a & 0x80) == 0) return tia_read(m, a);
    if ((a & 0x200) == 0) return m->ram[a & 0x7F];
    return riot_read(m, a);
}

static void beam_cycle(OMachine* m, uint64_t c);

/* The collision latches as a read during cycle c sees them: the pixels
   through colour clock 3c+2, the clocks of c included, as for a data read.
   The beam has passed the cycles before c; the rest is drawn on a copy of
   the machine (no frame buffer), so nothing here changes. */
static uint16_t latches_during(const OMachine* m, uint64_t c) {
    OMachine s = *m;
    s.fb = NULL;
    for (uint64_t k = s.beam_cycle; k <= c; k++) beam_cycle(&s, k);
    return s.cx;
}

/* instruction-fetch bus (also zero-page pointers), used at the first cycle
   of an instruction: the same map without side effects.  The cartridge area
   always shows ROM (the Superchip RAM window is for data only); a collision
   register shows its latches, which the TIA drives on every read of it. */
static uint8_t bus_peek(const OMachine* m, uint16_t addr) {
    uint16_t a = addr & 0x1FFF;
    if (a & 0x1000) return rom_byte(m, a);
    if ((a & 0x80) == 0)
        return (a & 0x0F) < 8 && m->track_cx ? tia_read_with(m, a, latches_during(m, m->beam_cycle))
                                             : tia_read(m, a);
    if ((a & 0x200) == 0) return m->ram[a & 0x7F];
    return riot_read(m, a);
}

static void bus_write(OMachine* m, uint16_t addr, uint8_t v) {
    uint16_t a = addr & 0x1FFF;
    if (a & 0x1000) { cart_write(m, a, v); return; }
    if ((a & 0x80) == 0) {
        /* 3F: a write to $00-$3F (not its mirrors) also picks the lower slice */
        if (m->scheme == SCH_3F && a <= 0x3F) m->bank = (uint16_t)(v % (m->rom_size / 2048));
        tia_write(m, a, v);
        return;
    }
    if ((a & 0x200) == 0) { m->ram[a & 0x7F] = v; return; }
    riot_write(m, a, v);
}

/* ------------------------------------------------------------------ video */

static int playfield_bit(const OMachine* m, int p) {
    if (p < 4) return (m->pf0 >> (4 + p)) & 1;          /* PF0 D4..D7 */
    if (p < 12) return (m->pf1 >> (7 - (p - 4))) & 1;   /* PF1 D7..D0 */
    return (m->pf2 >> (p - 12)) & 1;                    /* PF2 D0..D7 */
}

/* copies of a player / missile for NUSIZ mode 0-7: offsets, count */
static const uint8_t COPY_OFF[8][3] = {{0}, {0, 16}, {0, 32}, {0, 16, 32}, {0, 64}, {0}, {0, 32, 64}, {0}};
static const uint8_t COPY_N[8] = {1, 2, 2, 3, 2, 1, 3, 1};

static int player_on(uint8_t pos, uint8_t grp, uint8_t refp, uint8_t nusiz, int x) {
    int mode = nusiz & 7;
    int w = mode == 5 ? 2 : (mode == 7 ? 4 : 1);
    int d = (x - (int)pos + 160) % 160;
    for (int k = 0; k < COPY_N[mode]; k++) {
        int dd = d - COPY_OFF[mode][k];
        if (dd < 0 || dd >= 8 * w) continue;
        int b = dd / w;
        int bit = (refp & 8) ? b : 7 - b;
        return (grp >> bit) & 1;
    }
    return 0;
}

static int missile_on(uint8_t pos, uint8_t enam, uint8_t resmp, uint8_t nusiz, int x) {
    if (!(enam & 2) || (resmp & 2)) return 0;
    int mode = nusiz & 7;
    int size = 1 << ((nusiz >> 4) & 3);
    int n = (mode == 5 || mode == 7) ? 1 : COPY_N[mode];
    int d = (x - (int)pos + 160) % 160;
    for (int k = 0; k < n; k++) {
        int dd = d - COPY_OFF[mode][k];
        if (dd >= 0 && dd < size) return 1;
    }
    return 0;
}

static int ball_on(const OMachine* m, int x) {
    uint8_t en = (m->vdelbl & 1) ? m->enabl_old : m->enabl;
    if (!(en & 2)) return 0;
    int d = (x - (int)m->blx + 160) % 160;
    return d < (1 << ((m->ctrlpf >> 4) & 3));
}

/* the objects at visible pixel x: bit 0 PF, 1 BL, 2 P0, 3 P1, 4 M0, 5 M1 */
static int objects_at(const OMachine* m, int x) {
    int p;
    if (x < 80) p = x / 4;
    else if (m->ctrlpf & 1) p = 19 - (x - 80) / 4;
    else p = (x - 80) / 4;
    int o = playfield_bit(m, p);
    o |= ball_on(m, x) << 1;
    o |= player_on(m->p0x, (m->vdelp0 & 1) ? m->grp0_old : m->grp0, m->refp0, m->nusiz0, x) << 2;
    o |= player_on(m->p1x, (m->vdelp1 & 1) ? m->grp1_old : m->grp1, m->refp1, m->nusiz1, x) << 3;
    o |= missile_on(m->m0x, m->enam0, m->resmp0, m->nusiz0, x) << 4;
    o |= missile_on(m->m1x, m->enam1, m->resmp1, m->nusiz1, x) << 5;
    return o;
}

/* colour of pixel x (0..159) drawn with objects o */
static uint8_t pixel_colour(const OMachine* m, int x, int o) {
    int pf = o & 1, bl = (o >> 1) & 1, p0 = ((o >> 2) | (o >> 4)) & 1, p1 = ((o >> 3) | (o >> 5)) & 1;
    uint8_t pfc = (m->ctrlpf & 2) ? (x < 80 ? m->colup0 : m->colup1) : m->colupf;
    uint8_t fc = pf ? pfc : m->colupf;          /* the playfield/ball level */
    uint8_t c;
    if (m->ctrlpf & 4) {
        if (pf || bl) c = fc;
        else if (p0) c = m->colup0;
        else if (p1) c = m->colup1;
        else c = m->colubk;
    } else {
        if (p0) c = m->colup0;
        else if (p1) c = m->colup1;
        else if (pf || bl) c = fc;
        else c = m->colubk;
    }
    return (uint8_t)(c & 0xFE);
}

/* collision latches for objects o: (object a, object b, latch bit) */
static void collide(OMachine* m, int o) {
    static const uint8_t PAIRS[15][3] = {
        {4, 3, 1}, {4, 2, 0},     /* CXM0P:  M0-P1, M0-P0 */
        {5, 2, 3}, {5, 3, 2},     /* CXM1P:  M1-P0, M1-P1 */
        {2, 0, 5}, {2, 1, 4},     /* CXP0FB: P0-PF, P0-BL */
        {3, 0, 7}, {3, 1, 6},     /* CXP1FB: P1-PF, P1-BL */
        {4, 0, 9}, {4, 1, 8},     /* CXM0FB: M0-PF, M0-BL */
        {5, 0, 11}, {5, 1, 10},   /* CXM1FB: M1-PF, M1-BL */
        {1, 0, 13},               /* CXBLPF: BL-PF */
        {2, 3, 15}, {4, 5, 14}};  /* CXPPMM: P0-P1, M0-M1 */
    for (int i = 0; i < 15; i++)
        if (((o >> PAIRS[i][0]) & 1) && ((o >> PAIRS[i][1]) & 1)) m->cx |= (uint16_t)(1u << PAIRS[i][2]);
}

/* the beam during cycle c: colour clocks 3c .. 3c+2 */
static void beam_cycle(OMachine* m, uint64_t c) {
    if (!m->fb && !m->track_cx) return;
    for (int i = 0; i < 3; i++) {
        uint64_t g = 3 * c + (uint64_t)i;
        int64_t line = (int64_t)(g / 228);
        int h = (int)(g % 228);
        int64_t row = line - (int64_t)m->frame_line0 - 34;
        if (h < 68 || row < 0 || row >= 210) continue;
        int x = h - 68;
        uint8_t px = 0;
        if (!(m->vblank & 2) && !(x < 8 && line == m->hmove_blank_line)) {
            int o = objects_at(m, x);
            px = pixel_colour(m, x, o);
            if (m->track_cx) collide(m, o);
        }
        if (m->fb) m->fb[row * 160 + x] = px;
    }
}

static void full_cycle(OMachine* m, uint64_t c) {
    beam_cycle(m, c);
    timer_cycle(m);
}

/* -------------------------------------------------------------------- CPU */

static void set_nz(OMachine* m, uint8_t v) {
    m->p = (uint8_t)((m->p & ~(FL_N | FL_Z)) | (v & 0x80) | (v == 0 ? FL_Z : 0));
}

static void push(OMachine* m, uint8_t v) { bus_write(m, (uint16_t)(0x100 | m->sp), v); m->sp--; }
static uint8_t pull(OMachine* m) { m->sp++; return bus_read(m, (uint16_t)(0x100 | m->sp)); }

/* ADC, binary and NMOS decimal mode (B. Clark, "Decimal Mode", 6502.org,
   Appendix A: sequences 1 and 2; Z from the binary sum). */
static void op_adc(OMachine* m, uint8_t v) {
    int c = m->p & FL_C;
    int bin = m->a + v + c;
    if (!(m->p & FL_D)) {
        int ovf = (~(m->a ^ v) & (m->a ^ bin) & 0x80) != 0;
        m->p = (uint8_t)(m->p & ~(FL_C | FL_V));
        if (bin > 0xFF) m->p |= FL_C;
        if (ovf) m->p |= FL_V;
        m->a = (uint8_t)bin;
        set_nz(m, m->a);
        return;
    }
    int al = (m->a & 0x0F) + (v & 0x0F) + c;
    if (al >= 0x0A) al = ((al + 0x06) & 0x0F) + 0x10;
    int s = (m->a & 0xF0) + (v & 0xF0) + al;
    int sa = (int)(int8_t)(m->a & 0xF0) + (int)(int8_t)(v & 0xF0) + al;   /* signed */
    if (s >= 0xA0) s += 0x60;
    m->p = (uint8_t)(m->p & ~(FL_C | FL_V | FL_N | FL_Z));
    if (s >= 0x100) m->p |= FL_C;
    if (sa < -128 || sa > 127) m->p |= FL_V;
    if (sa & 0x80) m->p |= FL_N;
    if ((bin & 0xFF) == 0) m->p |= FL_Z;
    m->a = (uint8_t)s;
}

/* SBC: flags are always those of the binary subtraction; decimal mode
   changes only the accumulator (Clark, Appendix A, sequence 3). */
static void op_sbc(OMachine* m, uint8_t v) {
    int c = m->p & FL_C;
    int bin = m->a + (uint8_t)~v + c;
    int ovf = ((m->a ^ v) & (m->a ^ bin) & 0x80) != 0;
    uint8_t result;
    if (m->p & FL_D) {
        int al = (m->a & 0x0F) - (v & 0x0F) + c - 1;
        if (al < 0) al = ((al - 0x06) & 0x0F) - 0x10;
        int s = (m->a & 0xF0) - (v & 0xF0) + al;
        if (s < 0) s -= 0x60;
        result = (uint8_t)s;
    } else {
        result = (uint8_t)bin;
    }
    m->p = (uint8_t)(m->p & ~(FL_C | FL_V));
    if (bin > 0xFF) m->p |= FL_C;
    if (ovf) m->p |= FL_V;
    set_nz(m, (uint8_t)bin);
    m->a = result;
}

static void op_compare(OMachine* m, uint8_t reg, uint8_t v) {
    uint8_t d = (uint8_t)(reg - v);
    m->p = (uint8_t)(m->p & ~FL_C);
    if (reg >= v) m->p |= FL_C;
    set_nz(m, d);
}

/* ARR: A AND operand, rotated right through the carry.  Binary mode: N, Z
   from the result, C = bit 6, V = bit 6 XOR bit 5.  Decimal mode (NMOS): N
   is the incoming carry, Z from the rotated value, V = bit 6 changed by the
   rotate, then each nibble is BCD-corrected from the unrotated AND (low: +6
   when low nibble + its bit 0 exceeds 5; high: +$60 and C set when high
   nibble + its bit 4 exceeds $50, else C clear). */
static void op_arr(OMachine* m, uint8_t imm) {
    uint8_t t = (uint8_t)(m->a & imm);
    int cin = m->p & FL_C;
    uint8_t r = (uint8_t)((t >> 1) | (cin << 7));
    if (!(m->p & FL_D)) {
        m->a = r;
        set_nz(m, r);
        m->p = (uint8_t)(m->p & ~(FL_C | FL_V));
        if (r & 0x40) m->p |= FL_C;
        if (((r >> 6) ^ (r >> 5)) & 1) m->p |= FL_V;
        return;
    }
    m->p = (uint8_t)(m->p & ~(FL_N | FL_Z | FL_V | FL_C));
    if (cin) m->p |= FL_N;
    if (r == 0) m->p |= FL_Z;
    if ((t ^ r) & 0x40) m->p |= FL_V;
    if ((t & 0x0F) + (t & 0x01) > 5) r = (uint8_t)((r & 0xF0) | ((r + 6) & 0x0F));
    if ((t & 0xF0) + (t & 0x10) > 0x50) { r = (uint8_t)(r + 0x60); m->p |= FL_C; }
    m->a = r;
}

static int branch_taken(const OMachine* m, int mn) {
    switch (mn) {
    case BPL: return !(m->p & FL_N);
    case BMI: return (m->p & FL_N) != 0;
    case BVC: return !(m->p & FL_V);
    case BVS: return (m->p & FL_V) != 0;
    case BCC: return !(m->p & FL_C);
    case BCS: return (m->p & FL_C) != 0;
    case BNE: return !(m->p & FL_Z);
    case BEQ: return (m->p & FL_Z) != 0;
    }
    return 0;
}

static uint8_t shift_op(OMachine* m, int mn, uint8_t v) {
    uint8_t r = v;
    int cin = m->p & FL_C;
    switch (mn) {
    case ASL: m->p = (uint8_t)((m->p & ~FL_C) | ((v >> 7) & 1)); r = (uint8_t)(v << 1); break;
    case LSR: m->p = (uint8_t)((m->p & ~FL_C) | (v & 1)); r = (uint8_t)(v >> 1); break;
    case ROL: m->p = (uint8_t)((m->p & ~FL_C) | ((v >> 7) & 1)); r = (uint8_t)((v << 1) | cin); break;
    case ROR: m->p = (uint8_t)((m->p & ~FL_C) | (v & 1)); r = (uint8_t)((v >> 1) | (cin << 7)); break;
    case INC: r = (uint8_t)(v + 1); break;
    case DEC: r = (uint8_t)(v - 1); break;
    }
    set_nz(m, r);
    return r;
}

/*
 * Execute one instruction.  Returns 0, or END_VSYNC / END_CAP / END_ILLEGAL
 * when the frame ends with (or instead of) this instruction.
 */
int m_step_instruction(OMachine* m) {
    if (!table_ready) build_table();
    /* cycles the CPU spent halted by WSYNC */
    while (m->beam_cycle < m->cycle) full_cycle(m, m->beam_cycle++);
    uint64_t t = m->cycle;
    if (t / 76 >= m->frame_line0 + 320) { m->err |= 2; m->end_cycle = t - 1; return END_CAP; }

    uint8_t op = bus_peek(m, m->pc);
    uint8_t b1 = bus_peek(m, (uint16_t)(m->pc + 1));
    uint8_t b2 = bus_peek(m, (uint16_t)(m->pc + 2));
    Decoded d = DEC_TABLE[op];
    if (d.mn == ILL) { m->err |= 1; m->end_cycle = t - 1; return END_ILLEGAL; }

    int mn = d.mn, mode = d.mode;
    int len = 1;
    uint16_t ea = 0;
    int n = base_cycles(mn, mode);
    int cross = 0;
    switch (mode) {
    case IMP: case ACC: len = 1; break;
    case IMM: len = 2; break;
    case ZP: len = 2; ea = b1; break;
    case ZPX: len = 2; ea = (uint8_t)(b1 + m->x); break;
    case ZPY: len = 2; ea = (uint8_t)(b1 + m->y); break;
    case ABS: len = 3; ea = (uint16_t)(b1 | (b2 << 8)); break;
    case ABX: case ABY: {
        len = 3;
        uint16_t base = (uint16_t)(b1 | (b2 << 8));
        ea = (uint16_t)(base + (mode == ABX ? m->x : m->y));
        cross = (base & 0xFF00) != (ea & 0xFF00);
        break;
    }
    case IZX: {                        /* pointer in page zero, wraps within it */
        len = 2;
        uint8_t zp = (uint8_t)(b1 + m->x);
        ea = (uint16_t)(bus_peek(m, zp) | (bus_peek(m, (uint8_t)(zp + 1)) << 8));
        break;
    }
    case IZY: {
        len = 2;
        uint16_t base = (uint16_t)(bus_peek(m, b1) | (bus_peek(m, (uint8_t)(b1 + 1)) << 8));
        ea = (uint16_t)(base + m->y);
        cross = (base & 0xFF00) != (ea & 0xFF00);
        break;
    }
    case IND: len = 3; ea = (uint16_t)(b1 | (b2 << 8)); break;
    case REL: len = 2; break;
    }
    uint16_t next_pc = (uint16_t)(m->pc + len);
    uint16_t target = 0;
    int taken = 0;
    if (mode == REL) {
        taken = branch_taken(m, mn);
        target = (uint16_t)(next_pc + (int8_t)b1);
        if (taken) n += 1 + ((target & 0xFF00) != (next_pc & 0xFF00));
    } else if (cross && !is_store(mn) && !is_rmw(mn) && !is_combo(mn)) {
        n += 1;                        /* page-crossing penalty of indexed reads */
    }

    /* cycles t .. t+n-2, then the beam of the access cycle */
    for (uint64_t c = t; c < t + (uint64_t)n - 1; c++) full_cycle(m, c);
    uint64_t ac = t + (uint64_t)n - 1;
    beam_cycle(m, ac);
    m->access_cycle = ac;
    m->timer_written = 0;
    m->wsync_hit = 0;
    m->vsync_on = 0;

    m->pc = next_pc;
    uint8_t v;
    switch (mn) {
    case LDA: m->a = mode == IMM ? b1 : bus_read(m, ea); set_nz(m, m->a); break;
    case LDX: m->x = mode == IMM ? b1 : bus_read(m, ea); set_nz(m, m->x); break;
    case LDY: m->y = mode == IMM ? b1 : bus_read(m, ea); set_nz(m, m->y); break;
    case STA: bus_write(m, ea, m->a); break;
    case STX: bus_write(m, ea, m->x); break;
    case STY: bus_write(m, ea, m->y); break;
    case ADC: op_adc(m, mode == IMM ? b1 : bus_read(m, ea)); break;
    case SBC: op_sbc(m, mode == IMM ? b1 : bus_read(m, ea)); break;
    case AND: m->a &= mode == IMM ? b1 : bus_read(m, ea); set_nz(m, m->a); break;
    case ORA: m->a |= mode == IMM ? b1 : bus_read(m, ea); set_nz(m, m->a); break;
    case EOR: m->a ^= mode == IMM ? b1 : bus_read(m, ea); set_nz(m, m->a); break;
    case CMP: op_compare(m, m->a, mode == IMM ? b1 : bus_read(m, ea)); break;
    case CPX: op_compare(m, m->x, mode == IMM ? b1 : bus_read(m, ea)); break;
    case CPY: op_compare(m, m->y, mode == IMM ? b1 : bus_read(m, ea)); break;
    case BIT:
        v = bus_read(m, ea);
        m->p = (uint8_t)((m->p & ~(FL_N | FL_V | FL_Z)) | (v & (FL_N | FL_V)) | ((m->a & v) == 0 ? FL_Z : 0));
        break;
    case ASL: case LSR: case ROL: case ROR: case INC: case DEC:
        if (mode == ACC) m->a = shift_op(m, mn, m->a);
        else { v = bus_read(m, ea); bus_write(m, ea, shift_op(m, mn, v)); }
        break;
    case SLO: v = bus_read(m, ea); v = shift_op(m, ASL, v); bus_write(m, ea, v);
        m->a |= v; set_nz(m, m->a); break;
    case RLA: v = bus_read(m, ea); v = shift_op(m, ROL, v); bus_write(m, ea, v);
        m->a &= v; set_nz(m, m->a); break;
    case SRE: v = bus_read(m, ea); v = shift_op(m, LSR, v); bus_write(m, ea, v);
        m->a ^= v; set_nz(m, m->a); break;
    case RRA: v = bus_read(m, ea); v = shift_op(m, ROR, v); bus_write(m, ea, v);
        op_adc(m, v); break;                   /* the carry out of the rotate feeds the add */
    case DCP: v = bus_read(m, ea); v = (uint8_t)(v - 1); bus_write(m, ea, v);
        op_compare(m, m->a, v); break;
    case ISC: v = bus_read(m, ea); v = (uint8_t)(v + 1); bus_write(m, ea, v);
        op_sbc(m, v); break;
    case SAX: bus_write(m, ea, (uint8_t)(m->a & m->x)); break;
    case LAX: m->a = m->x = bus_read(m, ea); set_nz(m, m->a); break;
    case LAS: m->sp &= bus_read(m, ea); m->a = m->x = m->sp; set_nz(m, m->a); break;
    case ANC: m->a &= b1; set_nz(m, m->a); m->p = (uint8_t)((m->p & ~FL_C) | (m->a >> 7)); break;
    case ALR: m->a &= b1; m->p = (uint8_t)((m->p & ~FL_C) | (m->a & 1)); m->a >>= 1; set_nz(m, m->a); break;
    case ARR: op_arr(m, b1); break;
    case SBX: {
        uint8_t t = (uint8_t)(m->a & m->x);
        m->p = (uint8_t)((m->p & ~FL_C) | (t >= b1 ? FL_C : 0));
        m->x = (uint8_t)(t - b1);
        set_nz(m, m->x);
        break;
    }
    case INX: m->x++; set_nz(m, m->x); break;
    case INY: m->y++; set_nz(m, m->y); break;
    case DEX: m->x--; set_nz(m, m->x); break;
    case DEY: m->y--; set_nz(m, m->y); break;
    case TAX: m->x = m->a; set_nz(m, m->x); break;
    case TAY: m->y = m->a; set_nz(m, m->y); break;
    case TXA: m->a = m->x; set_nz(m, m->a); break;
    case TYA: m->a = m->y; set_nz(m, m->a); break;
    case TSX: m->x = m->sp; set_nz(m, m->x); break;
    case TXS: m->sp = m->x; break;
    case CLC: m->p &= (uint8_t)~FL_C; break;
    case SEC: m->p |= FL_C; break;
    case CLI: m->p &= (uint8_t)~FL_I; break;
    case SEI: m->p |= FL_I; break;
    case CLV: m->p &= (uint8_t)~FL_V; break;
    case CLD: m->p &= (uint8_t)~FL_D; break;
    case SED: m->p |= FL_D; break;
    case NOP: if (mode != IMP && mode != IMM) (void)bus_read(m, ea); break;   /* the read happens */
    case PHA: push(m, m->a); break;
    case PHP: push(m, (uint8_t)(m->p | FL_B | FL_U)); break;
    case PLA: m->a = pull(m); set_nz(m, m->a); break;
    case PLP: m->p = (uint8_t)((pull(m) & ~FL_B) | FL_U); break;
    case BPL: case BMI: case BVC: case BVS: case BCC: case BCS: case BNE: case BEQ:
        if (taken) m->pc = target;
        break;
    case JMP:
        if (mode == ABS) m->pc = ea;
        else {                         /* the pointer's high byte never leaves its page */
            uint8_t lo = bus_read(m, ea);
            uint8_t hi = bus_read(m, (uint16_t)((ea & 0xFF00) | ((ea + 1) & 0xFF)));
            m->pc = (uint16_t)(lo | (hi << 8));
        }
        break;
    case JSR: {
        uint16_t ret = (uint16_t)(next_pc - 1);   /* address of the JSR's last byte */
        push(m, (uint8_t)(ret >> 8));
        push(m, (uint8_t)ret);
        m->pc = ea;
        break;
    }
    case RTS: {
        uint8_t lo = pull(m);
        uint8_t hi = pull(m);
        m->pc = (uint16_t)((lo | (hi << 8)) + 1);
        break;
    }
    case RTI: {
        m->p = (uint8_t)((pull(m) & ~FL_B) | FL_U);
        uint8_t lo = pull(m);
        uint8_t hi = pull(m);
        m->pc = (uint16_t)(lo | (hi << 8));
        break;
    }
    case BRK: {
        uint16_t ret = (uint16_t)(m->pc + 1);     /* BRK skips a padding byte */
        push(m, (uint8_t)(ret >> 8));
        push(m, (uint8_t)ret);
        push(m, (uint8_t)(m->p | FL_B | FL_U));
        m->p |= FL_I;
        uint8_t lo = bus_read(m, 0xFFFE);
        uint8_t hi = bus_read(m, 0xFFFF);
        m->pc = (uint16_t)(lo | (hi << 8));
        break;
    }
    default: break;
    }

    if (!m->timer_written) timer_cycle(m);
    m->beam_cycle = ac + 1;
    m->cycle = ac + 1;
    m->instr_count++;
    if (m->wsync_hit) m->cycle = 76 * (ac / 76 + 1);
    if (m->vsync_on) {
        m->end_cycle = ac;
        m->frame_line0 = ac / 76;
        return END_VSYNC;
    }
    return 0;
}

/* Run until the frame ends.  `fb` (210 x 160) receives the frame if non-NULL. */
int m_run_frame(OMachine* m, uint8_t* fb, uint64_t* end_cycle) {
    m->fb = fb;
    if (fb) memset(fb, 0, 210 * 160);
    int why;
    for (;;) {
        why = m_step_instruction(m);
        if (why) break;
    }
    /* a capped or faulted frame ends before the instruction that could not start */
    if (why != END_VSYNC) m->frame_line0 = m->end_cycle / 76;
    if (end_cycle) *end_cycle = m->end_cycle;
    m->fb = NULL;
    return why;
}

/* Joystick and button of player 0 for one of the 18 actions (ALE order). */
void m_set_action(OMachine* m, uint32_t action) {
    /* bits: 1 up, 2 down, 4 left, 8 right, 16 fire */
    static const uint8_t map[18] = {
        0, 16, 1, 8, 4, 2, 1 | 8, 1 | 4, 2 | 8, 2 | 4,
        1 | 16, 8 | 16, 4 | 16, 2 | 16, 1 | 8 | 16, 1 | 4 | 16, 2 | 8 | 16, 2 | 4 | 16};
    uint8_t b = action < 18 ? map[action] : 0;
    uint8_t up = b & 1, down = (b >> 1) & 1, left = (b >> 2) & 1, right = (b >> 3) & 1;
    /* SWCHA high nibble, active low: D7 right, D6 left, D5 down, D4 up */
    uint8_t pressed = (uint8_t)((right << 7) | (left << 6) | (down << 5) | (up << 4));
    m->swcha = (uint8_t)(~pressed);
    m->swcha |= 0x0F;                  /* player 1 idle */
    m->inpt4 = (b & 16) ? 0x00 : 0x80;
}

void m_power_on(OMachine* m, const uint8_t* rom, uint32_t size, uint32_t scheme) {
    memset(m, 0, sizeof(*m));
    m->rom = rom;
    m->rom_size = size;
    m->scheme = scheme;
    if (scheme == SCH_E0) m->bank = 4 | (5 << 3) | (6 << 6);
    else if (scheme == SCH_3F) m->bank = 0;
    else m->bank = (uint16_t)(linear_banks(scheme) - 1);     /* the last 4 KB bank */
    m->sp = 0xFD;
    m->p = 0x24;
    m->tim_interval = 1024;            /* INTIM reads 0 from cycle 0, interval 1024 */
    m->hmove_blank_line = -1;
    m->pc = (uint16_t)(rom_byte(m, 0x1FFC) | (rom_byte(m, 0x1FFD) << 8));
    m_set_action(m, 0);
}

/* ---------------------------------------------------------- state record */

static void put16(uint8_t* p, uint16_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
static void put32(uint8_t* p, uint32_t v) { for (int i = 0; i < 4; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static void put64(uint8_t* p, uint64_t v) { for (int i = 0; i < 8; i++) p[i] = (uint8_t)(v >> (8 * i)); }
static uint16_t get16(const uint8_t* p) { return (uint16_t)(p[0] | (p[1] << 8)); }
static uint32_t get32(const uint8_t* p) { uint32_t v = 0; for (int i = 3; i >= 0; i--) v = (v << 8) | p[i]; return v; }
static uint64_t get64(const uint8_t* p) { uint64_t v = 0; for (int i = 7; i >= 0; i--) v = (v << 8) | p[i]; return v; }

void m_to_record(const OMachine* src, uint8_t* out) {
    OMachine m = *src;
    /* the timer as a read at `cycle` would see it (advance over a WSYNC halt) */
    while (m.beam_cycle < m.cycle) { timer_cycle(&m); m.beam_cycle++; }
    memset(out, 0, 384);
    out[0] = m.a; out[1] = m.x; out[2] = m.y; out[3] = m.sp; out[4] = m.p; out[5] = (uint8_t)m.bank;
    out[31] = (uint8_t)(m.bank >> 8);
    put16(out + 6, m.pc);
    put64(out + 8, m.cycle);
    put64(out + 16, m.frame_line0);
    out[24] = m.tim_count;
    out[25] = m.tim_expired;
    put16(out + 26, m.tim_interval);
    put16(out + 28, m.tim_expired ? 0 : m.tim_sub);
    memcpy(out + 32, m.ram, 128);
    const uint8_t regs[18] = {m.vsync, m.vblank, m.colup0, m.colup1, m.colupf, m.colubk, m.ctrlpf,
                              m.refp0, m.refp1, m.pf0, m.pf1, m.pf2, m.grp0, m.grp1, m.hmp0, m.hmp1,
                              m.p0x, m.p1x};
    memcpy(out + 160, regs, 18);
    put32(out + 180, m.rom_id);
    put32(out + 184, m.step_idx);
    put32(out + 188, m.episode_idx);
    out[192] = m.prev_action;
    out[194] = m.err;
    put64(out + 200, m.instr_count);
    const uint8_t objs[19] = {m.nusiz0, m.nusiz1, m.enam0, m.enam1, m.enabl, m.enabl_old, m.grp0_old, m.grp1_old,
                              m.vdelp0, m.vdelp1, m.vdelbl, m.resmp0, m.resmp1, m.m0x, m.m1x, m.blx,
                              m.hmm0, m.hmm1, m.hmbl};
    memcpy(out + 208, objs, 19);
    out[227] = m.hmove_blank_line == (int64_t)(m.cycle / 76);
    put16(out + 228, m.cx);
    out[230] = m.track_cx;
    memcpy(out + 256, m.xram, 128);
}

void m_from_record(OMachine* m, const uint8_t* in) {
    m->a = in[0]; m->x = in[1]; m->y = in[2]; m->sp = in[3]; m->p = in[4];
    m->bank = (uint16_t)(in[5] | (in[31] << 8));
    m->pc = get16(in + 6);
    m->cycle = get64(in + 8);
    m->beam_cycle = m->cycle;
    m->frame_line0 = get64(in + 16);
    m->tim_count = in[24];
    m->tim_expired = in[25];
    m->tim_interval = get16(in + 26);
    m->tim_sub = get16(in + 28);
    memcpy(m->ram, in + 32, 128);
    const uint8_t* r = in + 160;
    m->vsync = r[0]; m->vblank = r[1]; m->colup0 = r[2]; m->colup1 = r[3]; m->colupf = r[4];
    m->colubk = r[5]; m->ctrlpf = r[6]; m->refp0 = r[7]; m->refp1 = r[8]; m->pf0 = r[9];
    m->pf1 = r[10]; m->pf2 = r[11]; m->grp0 = r[12]; m->grp1 = r[13]; m->hmp0 = r[14];
    m->hmp1 = r[15]; m->p0x = r[16]; m->p1x = r[17];
    m->rom_id = get32(in + 180);
    m->step_idx = get32(in + 184);
    m->episode_idx = get32(in + 188);
    m->prev_action = in[192];
    m->err = in[194];
    m->instr_count = get64(in + 200);
    const uint8_t* o = in + 208;
    m->nusiz0 = o[0]; m->nusiz1 = o[1]; m->enam0 = o[2]; m->enam1 = o[3]; m->enabl = o[4]; m->enabl_old = o[5];
    m->grp0_old = o[6]; m->grp1_old = o[7]; m->vdelp0 = o[8]; m->vdelp1 = o[9]; m->vdelbl = o[10];
    m->resmp0 = o[11]; m->resmp1 = o[12]; m->m0x = o[13]; m->m1x = o[14]; m->blx = o[15];
    m->hmm0 = o[16]; m->hmm1 = o[17]; m->hmbl = o[18];
    m->hmove_blank_line = in[227] ? (int64_t)(m->cycle / 76) : -1;
    m->cx = get16(in + 228);
    m->track_cx = in[230];
    memcpy(m->xram, in + 256, 128);
}
