"""Test helpers: machine-state record decoding and small program harnesses."""
import numpy as np

from paper_1907_08467_amd.inputs.asm6502 import assemble, assemble_with_symbols

TIA_NAMES = ["VSYNC", "VBLANK", "COLUP0", "COLUP1", "COLUPF", "COLUBK", "CTRLPF", "REFP0", "REFP1",
             "PF0", "PF1", "PF2", "GRP0", "GRP1", "HMP0", "HMP1", "P0X", "P1X"]


def u16(rec, o):
    return int(rec[o]) | (int(rec[o + 1]) << 8)


def u32(rec, o):
    return int.from_bytes(bytes(rec[o:o + 4]), "little")


def u64(rec, o):
    return int.from_bytes(bytes(rec[o:o + 8]), "little")


def decode(rec):
    rec = np.asarray(rec, dtype=np.uint8)
    d = dict(a=int(rec[0]), x=int(rec[1]), y=int(rec[2]), sp=int(rec[3]), p=int(rec[4]), bank=int(rec[5]) | (int(rec[31]) << 8),
             pc=u16(rec, 6), cycle=u64(rec, 8), frame_line0=u64(rec, 16), intim=int(rec[24]),
             expired=int(rec[25]), interval=u16(rec, 26), phase=u16(rec, 28), ram=rec[32:160].copy(),
             rom_id=u32(rec, 180), step_idx=u32(rec, 184), episode_idx=u32(rec, 188),
             prev_action=int(rec[192]), err=int(rec[194]), instr=u64(rec, 200),
             xram=rec[256:384].copy())
    for i, n in enumerate(TIA_NAMES):
        d[n] = int(rec[160 + i])
    return d


def set_fields(rec, **kw):
    rec = np.array(rec, dtype=np.uint8, copy=True)
    off1 = dict(a=0, x=1, y=2, sp=3, p=4)
    for k, v in kw.items():
        if k in off1:
            rec[off1[k]] = v
        elif k == "bank":
            rec[5], rec[31] = v & 0xFF, v >> 8
        elif k == "pc":
            rec[6], rec[7] = v & 0xFF, v >> 8
        elif k == "cycle":
            rec[8:16] = np.frombuffer(int(v).to_bytes(8, "little"), dtype=np.uint8)
        elif k == "ram":
            for addr, val in v.items():
                rec[32 + (addr & 0x7F)] = val
        elif k.upper() in TIA_NAMES:
            rec[160 + TIA_NAMES.index(k.upper())] = v
        else:
            raise KeyError(k)
    return rec


def diff_records(a, b):
    """Human-readable list of differing fields between two state records."""
    da, db = decode(a), decode(b)
    out = []
    for k in da:
        va, vb = da[k], db[k]
        if isinstance(va, np.ndarray):
            idx = np.nonzero(va != vb)[0]
            if idx.size:
                out.append(f"{k}[{[hex(0x80 + int(i)) for i in idx[:8]]}]: {va[idx[:8]]} vs {vb[idx[:8]]}")
        elif va != vb:
            out.append(f"{k}: {va} vs {vb}")
    return out


def cart(src, banks=1):
    """Assemble a 4 KB test cartridge; `src` must define the label `reset`.
    The reset and BRK vectors are added at $1FFC-$1FFF unless `src` sets them."""
    if ".org $1FFC" not in src:
        src += "\n    .org $1FFC\n    .word reset\n    .word reset\n"
    return assemble_with_symbols(src, banks=banks)
