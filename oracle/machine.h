/* Internal declarations of the CPU oracle (test infrastructure). */
#ifndef VCS_ORACLE_MACHINE_H
#define VCS_ORACLE_MACHINE_H

#include <stdint.h>

/* status flags */
#define FL_C 0x01
#define FL_Z 0x02
#define FL_I 0x04
#define FL_D 0x08
#define FL_B 0x10
#define FL_U 0x20
#define FL_V 0x40
#define FL_N 0x80

typedef struct {
    /* cartridge */
    const uint8_t* rom;
    uint32_t rom_size;
    uint32_t scheme;            /* SCH_* below */
    uint16_t bank;              /* bank state: 4 KB bank (4K/F8/F6/F4 and their
                                   Superchip forms), E0 slices s0 | s1 << 3 | s2 << 6,
                                   or the 3F slice of the lower 2 KB */
    uint8_t xram[128];          /* Superchip RAM */
    /* 6507 */
    uint8_t a, x, y, sp, p;
    uint16_t pc;
    uint64_t cycle;             /* start cycle of the next instruction */
    uint64_t beam_cycle;        /* first cycle the beam and timer have not yet passed */
    uint64_t instr_count;
    /* RIOT */
    uint8_t ram[128];
    uint8_t tim_count;
    uint8_t tim_expired;
    uint16_t tim_sub;
    uint16_t tim_interval;
    /* TIA write registers (last byte written) and object positions */
    uint8_t vsync, vblank, colup0, colup1, colupf, colubk, ctrlpf, refp0, refp1;
    uint8_t pf0, pf1, pf2, grp0, grp1, hmp0, hmp1;
    uint8_t p0x, p1x;
    uint8_t nusiz0, nusiz1, enam0, enam1, enabl, resmp0, resmp1;
    uint8_t vdelp0, vdelp1, vdelbl, hmm0, hmm1, hmbl;
    uint8_t grp0_old, grp1_old, enabl_old;     /* the vertical-delay copies */
    uint8_t m0x, m1x, blx;
    int64_t hmove_blank_line;   /* line whose pixels 0-7 an early HMOVE blanked, or -1 */
    uint16_t cx;                /* collision latches: bit 2r+1 = D7, bit 2r = D6 of CX register r */
    uint8_t track_cx;           /* collision latches tracked (else they read 0) */
    /* the frame being emulated */
    uint64_t frame_line0;
    uint8_t* fb;                /* 210 x 160 frame buffer, or NULL */
    /* console inputs of the current frame */
    uint8_t swcha, inpt4;
    /* env bookkeeping */
    uint32_t rom_id, step_idx, episode_idx;
    uint8_t prev_action, err;
    /* per-instruction scratch */
    uint64_t access_cycle;
    uint64_t end_cycle;         /* last cycle of the frame that just ended */
    int timer_written, wsync_hit, vsync_on;
} OMachine;

/* cartridge schemes */
#define SCH_4K 0
#define SCH_F8 1
#define SCH_F6 2
#define SCH_F4 3
#define SCH_F8SC 4
#define SCH_F6SC 5
#define SCH_F4SC 6
#define SCH_E0 7
#define SCH_3F 8
#define SCH_COUNT 9

/* frame end reasons */
#define END_VSYNC 1
#define END_CAP 2
#define END_ILLEGAL 3

int m_rom_size_ok(uint32_t size, uint32_t scheme);
void m_power_on(OMachine* m, const uint8_t* rom, uint32_t size, uint32_t scheme);
int m_step_instruction(OMachine* m);      /* 0 or an END_* code */
int m_run_frame(OMachine* m, uint8_t* fb, uint64_t* end_cycle);
void m_set_action(OMachine* m, uint32_t action);
void m_to_record(const OMachine* m, uint8_t* out);
void m_from_record(OMachine* m, const uint8_t* in);

#endif
