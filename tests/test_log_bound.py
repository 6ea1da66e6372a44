"""The row log's capacity against the densest TIA writing a program can do.

Each emulated TIA write logs at most one entry in the row its effect lands
in.  All data accesses of an instruction happen at its last cycle, and a
write at access cycle c takes effect at colour clock 3(c+1), visible when
that clock is 68..227 of its line.  So the entries of one row come from the
instructions whose access cycles fall in one window of visible cycles: the
first of them may have started earlier, every later one adds its whole
length.  The bound is the most writes such a sequence makes, from the
datasheet cycle counts (documented and stable undocumented opcodes) and the
writes each instruction makes (stores, read-modify-write, pushes: JSR 2, BRK
3).  The library's row and frame capacities must hold it, plus the one
frame-end entry.
"""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))

ONE_WRITE = {"STA", "STX", "STY", "SAX", "PHA", "PHP", "SLO", "RLA", "SRE", "RRA", "DCP", "ISC"}
RMW = {"ASL", "LSR", "ROL", "ROR", "INC", "DEC"}


def opcode_rows():
    for name in ("mos6502_opcodes.txt", "nmos6502_undocumented.txt"):
        for line in open(os.path.join(HERE, "golden", name)):
            if line.startswith("#") or not line.strip():
                continue
            op, mn, mode, _nbytes, cyc = line.split()[:5]
            if cyc == "fault":
                continue
            yield mn, mode, int(cyc.split("+")[0])


def writes(mn, mode):
    if mn == "BRK":
        return 3
    if mn == "JSR":
        return 2
    if mn in ONE_WRITE or (mn in RMW and mode != "acc"):
        return 1
    return 0


def visible_window():
    """Access cycles of a line whose write lands in the visible part."""
    return sum(1 for c in range(76) if 3 * ((c + 1) % 76) >= 68)


def row_bound():
    kinds = {(cyc, writes(mn, mode)) for mn, mode, cyc in opcode_rows()}
    span = visible_window() - 1           # cycles after the first access cycle in the window
    best = [0] * (span + 1)               # unbounded knapsack: most writes within `cap` cycles
    for cap in range(1, span + 1):
        best[cap] = max([best[cap - 1]] + [best[cap - n] + w for n, w in kinds if n <= cap])
    return max(w for _, w in kinds) + best[span]


def header_consts():
    src = open(os.path.join(ROOT, "paper_1907_08467_amd", "csrc", "vcs_device.h")).read()
    out = {}
    for name in ("kRows", "kRowEntries", "kSnapBytes", "kSnapArea", "kFrameEntries"):
        out[name] = int(re.search(rf"constexpr int {name} = (\d+);", src).group(1))
    out["kCountMask"] = int(re.search(r"constexpr uint32_t kCountMask = (0x[0-9A-Fa-f]+);", src).group(1), 16)
    return out


def test_visible_window_is_53_cycles():
    assert visible_window() == 53


def test_densest_row_is_eight_brk_and_a_store():
    # BRK at the window's first cycle, seven more 7-cycle BRKs (49 cycles)
    # and one 3-cycle store in the 52 cycles after it
    assert row_bound() == 3 + 7 * 3 + 1 == 25


def test_log_capacity_holds_the_bound():
    k = header_consts()
    bound = row_bound()
    assert k["kRowEntries"] >= bound
    assert k["kCountMask"] >= bound + 1                       # the row count field, frame end included
    assert k["kFrameEntries"] >= k["kRows"] * bound + 1       # the whole frame's stream
    assert k["kSnapArea"] >= k["kRows"] * k["kSnapBytes"]
    assert k["kSnapArea"] % 128 == 0 and k["kFrameEntries"] % 32 == 0
