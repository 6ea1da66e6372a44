"""Every cartridge scheme and the undocumented opcodes on the GPU against
the oracle: fuzz cartridges (hotspots, Superchip ports, E0/3F slice
switching, instructions straddling a segment boundary, the stable
undocumented opcodes in every addressing mode) stepped on both sides with
the same actions; full machine-state records compared every step.  A mixed
batch puts one ROM of every scheme into a single launch (the wide-ROM
interpreter, 32 KB of cartridge in LDS) next to the plain 4 KB workload ROM.
"""
import sys

import numpy as np
import pytest

from fuzzcart import S_3F, S_E0, S_F4, S_F4SC, S_F6, S_F6SC, S_F8, S_F8SC, S_4K, fuzz_cart
from helpers import diff_records
from parity import make_pair, step_both
from paper_1907_08467_amd.inputs.romgen import RomSpec, generate

pytestmark = pytest.mark.gpu

CASES = [(S_4K, True, 4096), (S_F8, True, 8192), (S_F6, False, 0), (S_F6, True, 0), (S_F4, True, 0),
         (S_F8SC, False, 0), (S_F8SC, True, 0), (S_F6SC, True, 0), (S_F4SC, True, 0), (S_E0, False, 0),
         (S_E0, True, 0), (S_3F, False, 8192), (S_3F, True, 4096), (S_3F, True, 32768)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare_all(o, g, n, tag):
    for e in range(n):
        a, b = g.get_state(e), o.get_state(e)
        assert np.array_equal(a, b), f"{tag}: env {e}: {diff_records(a, b)}"


@pytest.mark.parametrize("scheme,undoc,size", CASES, ids=[f"s{c[0]}_u{int(c[1])}_{c[2]}" for c in CASES])
def test_fuzz_scheme(scheme, undoc, size):
    seed = 2000 + 17 * scheme + (1 if undoc else 0) + size // 4096
    say(f"case: scheme {scheme} undoc {undoc} size {size} seed {seed}")
    rom, sch = fuzz_cart(seed, scheme=scheme, undoc=undoc, size=size or 8192)
    n = 40
    o, g = make_pair([(rom, sch)], np.zeros(n, np.uint16), seed=seed, frameskip=2 + seed % 3)
    rng = np.random.default_rng(seed)
    for s in range(25):
        step_both(o, g, rng.integers(0, 18, n), want_frames=True, tag=f"scheme {scheme} step {s}")
        compare_all(o, g, n, f"scheme {scheme} step {s}")
    assert g.poll_errors() == o.poll_errors()
    g.close()
    o.close()


def test_mixed_scheme_batch():
    """One launch over ROMs of every scheme (tiles by ROM), listed ids."""
    roms = [(generate(RomSpec(1000)).data, 0)]
    for k, (sch, size) in enumerate([(S_F8, 0), (S_F6SC, 0), (S_F4, 0), (S_E0, 0), (S_3F, 16384), (S_4K, 0)]):
        roms.append(fuzz_cart(3000 + k, scheme=sch, undoc=True, size=size or 8192))
    n = 7 * 24
    env_rom = (np.arange(n) % 7).astype(np.uint16)
    say(f"case: mixed scheme batch, {n} envs over {len(roms)} ROMs")
    o, g = make_pair(roms, env_rom, seed=9, frameskip=4)
    rng = np.random.default_rng(9)
    for s in range(16):
        ids = np.sort(rng.permutation(n)[:150]).astype(np.int32) if s % 2 else None
        m = n if ids is None else ids.size
        step_both(o, g, rng.integers(0, 18, m), ids=ids, want_frames=s % 4 == 0, tag=f"mixed step {s}")
    compare_all(o, g, n, "mixed")
    assert g.poll_errors() == o.poll_errors()
    g.close()
    o.close()


def test_bank_state_validation():
    rom, sch = fuzz_cart(4000, scheme=S_3F, size=8192)
    o, g = make_pair([(rom, sch)], np.zeros(2, np.uint16))
    rec = g.get_state(0)
    bad = rec.copy()
    bad[5] = 4                                    # 3F with 4 slices: bank state 0..3
    from paper_1907_08467_amd import binding as B
    with pytest.raises(B.VcsError):
        g.set_state(0, bad)
    ok = rec.copy()
    ok[5] = 3
    g.set_state(0, ok)
    assert g.get_state(0)[5] == 3
    g.close()
    o.close()
