"""The seeded input generators: determinism, sizes and the stated structure."""
import numpy as np

from paper_2406_18111_amd import synth


def test_splitmix_reference_values():
    # SplitMix64 with state 0: first outputs as published with the generator
    s = synth.Stream.__new__(synth.Stream)
    s.base, s.pos = 0, 0
    got = [int(x) for x in s.raw(3)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_config0_shape_and_structure():
    t, m = synth.config0()
    t2, _ = synth.config0()
    assert m == 8 and t.dtype == np.uint64 and len(t) == 4096
    assert np.array_equal(t, t2)
    # loop body of 50: most positions equal the one 50 earlier
    same = np.mean(t[50:] == t[:-50])
    assert 0.85 < same < 0.95


def test_config1_shape():
    t, m = synth.config1(n=1 << 16)
    assert m == 16 and len(t) == 1 << 16 and t.dtype == np.uint64
    assert np.array_equal(t, synth.config1(n=1 << 16)[0])
    # prefix property: a longer draw starts with the shorter one
    assert np.array_equal(synth.config1(n=1 << 17)[0][: 1 << 16], t)


def test_config2_shape():
    t, m = synth.config2(n=1 << 12)
    assert m == 32 and t.dtype == np.uint32
    assert not t[: 1 << 11].any()
    assert set(np.unique(t[1 << 11:]).tolist()) <= {0, 1, 2, 3}


def test_config3_lengths():
    wins, m = synth.config3(num_windows=64)
    assert m == 8 and len(wins) == 64
    lens = [len(w) for w in wins]
    assert min(lens) >= 256 and max(lens) <= 65536


def test_config4_trace():
    reqs = list(synth.config4_trace(duration=0.05))
    assert len(reqs) > 20
    assert all(1024 <= len(r.tokens) <= 1 << 20 for r in reqs)
    assert all(reqs[i].arrival < reqs[i + 1].arrival for i in range(len(reqs) - 1))
