"""The seeded generators: pinned to their published definitions and to the
statistics of the workload recipes (no GPU)."""
import numpy as np

import synth

M64 = (1 << 64) - 1


def _splitmix64(x):
    x = (x + 0x9E3779B97F4A7C15) & M64
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return x, z ^ (z >> 31)


def _rotl(x, k):
    return ((x << k) | (x >> (64 - k))) & M64


def test_xoshiro256starstar_matches_its_definition():
    seed = 12345
    s, x = [], seed
    for _ in range(4):
        x, z = _splitmix64(x)
        s.append(z)
    want = []
    for _ in range(50):
        want.append((_rotl((s[1] * 5) & M64, 7) * 9) & M64)
        t = (s[1] << 17) & M64
        s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3]
        s[2] ^= t
        s[3] = _rotl(s[3], 45)
    assert synth.raw_u64(seed, 50).tolist() == want


def test_iid_composition():
    g = synth.iid(synth.substream(1, 0), 1 << 20, 0.01)
    assert set(np.unique(g).tolist()) <= set(b"ACGTN")
    frac_n = np.mean(g == ord("N"))
    assert abs(frac_n - 0.01) < 0.001
    for ch in b"ACGT":
        assert abs(np.mean(g == ch) - 0.2475) < 0.003


def test_markov_genome_decorations():
    g, offs = synth.workload_markov_batch(n_seqs=256, seq_len=8192, seed=77)
    assert offs[-1] == g.size == 256 * 8192
    lower = np.isin(g, np.frombuffer(b"acgtn", np.uint8))
    n_frac = np.mean(np.isin(g, np.frombuffer(b"Nn", np.uint8)))
    invalid = ~np.isin(g, np.frombuffer(b"ACGTNacgtn", np.uint8))
    assert abs(lower.mean() - 0.40) < 0.05
    assert abs(n_frac - 0.02) < 0.008
    assert 0.3e-4 < invalid.mean() < 2.5e-4


def _cond_entropy(seq, order):
    d = np.frombuffer(seq.tobytes().translate(bytes.maketrans(b"ACGT", b"\x00\x01\x02\x03")), np.uint8).astype(np.int64)
    ctx = np.zeros(d.size - order, dtype=np.int64)
    for j in range(order):
        ctx = ctx * 4 + d[j:d.size - order + j]
    nxt = d[order:]
    joint = np.bincount(ctx * 4 + nxt, minlength=4 ** (order + 1)).reshape(-1, 4).astype(float)
    p_ctx = joint.sum(1, keepdims=True)
    with np.errstate(divide="ignore", invalid="ignore"):
        h = -np.nansum(joint / joint.sum() * np.log2(joint / p_ctx))
    return h


def test_markov_order_is_visible_in_conditional_entropy():
    g = synth.markov(synth.substream(2, 1), 99, 3, 1 << 21)
    h2, h3, h4 = (_cond_entropy(g, m) for m in (2, 3, 4))
    assert h3 < h2 - 0.02          # the 3rd base back carries information
    assert abs(h4 - h3) < 0.01     # the 4th does not


def test_generators_are_deterministic():
    a = synth.workload_markov_batch(n_seqs=8, seq_len=1000, seed=5)[0]
    b = synth.workload_markov_batch(n_seqs=8, seq_len=1000, seed=5)[0]
    c = synth.workload_markov_batch(n_seqs=8, seq_len=1000, seed=6)[0]
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_chromosome_lengths_sum_to_two_gib():
    lens = synth.chromosome_lengths()
    assert lens.size == 16 and int(lens.sum()) == 1 << 31 and lens.min() > 0


def test_bpe_batch_lengths_and_trace():
    _, offs = synth.workload_bpe_batch(n_seqs=1024)
    lens = np.diff(offs)
    assert lens.min() >= 500 and lens.max() < 20000
    assert 4.5e6 < offs[-1] < 6.5e6
    arr, sizes, vocab = synth.serving_trace(n_requests=20000)
    gaps = np.diff(arr)
    assert abs(gaps.mean() - 1 / 2000) < 5e-5
    assert sizes.min() >= 100 and sizes.max() < 1_000_000
    assert set(np.unique(vocab).tolist()) == {0, 1, 2, 3}
