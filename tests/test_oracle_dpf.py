"""Pins for the oracle's DPF (paper section 3.1, Eq. (p1)-(p3)) and PIR answer.

Each check is fixed by the paper or by mathematics, not by the oracle itself:
  - the DPF identity Eval(k_a, j) + Eval(k_b, j) = beta * [j == alpha], by brute
    force over every j (and every alpha on small domains);
  - the node structure the construction must have at every depth (off-path
    nodes equal across the two parties, on-path control bits different), which
    also fixes the parent map floor(j / 2) of the paper's L = 4 walk-through;
  - the work counts the paper states: O(L) PRF calls for full evaluation
    (exactly 2(L - 1)), O(log L) for Gen;
  - the key sizes printed in Table 4;
  - the PIR identity T x (Eval_a + Eval_b) = T[alpha], and the per-server
    answer recomputed by an independent numpy product mod 2^32.
"""
import numpy as np
import pytest

from conftest import read_golden

BETAS = [0, 1, 2, 2**31, 2**32 - 1, 0x9E3779B9]


def seed_for(*ints) -> bytes:
    rng = np.random.default_rng(list(ints))
    return rng.integers(0, 256, 16, dtype=np.uint8).tobytes()


def indicator(n, alpha, beta):
    e = np.zeros(1 << n, np.uint32)
    e[alpha] = beta & 0xFFFFFFFF
    return e


@pytest.mark.parametrize("n", range(1, 7))
def test_dpf_identity_every_alpha(O, n):
    for alpha in range(1 << n):
        beta = BETAS[alpha % len(BETAS)]
        k0, k1 = O.gen(n, alpha, beta, seed_for(n, alpha))
        s = O.eval_full(k0) + O.eval_full(k1)
        assert (s.astype(np.uint32) == indicator(n, alpha, beta)).all(), (n, alpha)


@pytest.mark.parametrize("n", [7, 8, 9, 10, 12])
@pytest.mark.parametrize("beta", BETAS)
def test_dpf_identity_random_alpha(O, n, beta):
    rng = np.random.default_rng([n, beta])
    for trial in range(3):
        alpha = int(rng.integers(0, 1 << n))
        k0, k1 = O.gen(n, alpha, beta, seed_for(n, beta, trial))
        s = (O.eval_full(k0) + O.eval_full(k1)).astype(np.uint32)
        assert (s == indicator(n, alpha, beta)).all()


def test_extreme_alphas_and_domains(O):
    for n in (1, 2, 16):
        for alpha in (0, (1 << n) - 1):
            k0, k1 = O.gen(n, alpha, 1, seed_for(99, n, alpha))
            s = (O.eval_full(k0) + O.eval_full(k1)).astype(np.uint32)
            assert (s == indicator(n, alpha, 1)).all()


def test_point_eval_matches_full_eval(O):
    n, alpha = 9, 300
    k0, k1 = O.gen(n, alpha, 5, seed_for(5))
    for key in (k0, k1):
        full = O.eval_full(key)
        for j in (0, 1, 2, 255, 299, 300, 301, 511):
            assert O.eval_point(key, j) == full[j]


def test_large_domain_point_identity(O):
    """n = 32: full evaluation is out of reach, point evaluation is not."""
    n = 32
    alpha = 0xDEADBEEF
    k0, k1 = O.gen(n, alpha, 77, seed_for(32))
    for j in (alpha, alpha - 1, alpha + 1, 0, 2**32 - 1, alpha ^ (1 << 31)):
        got = (O.eval_point(k0, j) + O.eval_point(k1, j)) & 0xFFFFFFFF
        assert got == (77 if j == alpha else 0)


def tbit(seed_row):
    return int(seed_row[0]) & 1


@pytest.mark.parametrize("n,alpha,beta", [(6, 45, 1), (8, 0, 2**31), (8, 255, 7), (10, 613, 0)])
def test_node_invariants(O, n, alpha, beta):
    """At depth d the on-path node is floor(alpha / 2^(n-d)) (parent of (d, j) is
    (d-1, floor(j/2))).  Off-path seeds agree between the parties; on-path
    control bits differ above the leaves; the on-path leaves differ by beta."""
    k0, k1 = O.gen(n, alpha, beta, seed_for(n, alpha, beta))
    for d in range(0, n + 1):
        L0, L1 = O.eval_level(k0, d), O.eval_level(k1, d)
        on = alpha >> (n - d)
        for j in range(1 << d):
            if j != on:
                assert (L0[j] == L1[j]).all(), (d, j)
        if d < n:
            assert tbit(L0[on]) != tbit(L1[on]), d
        else:
            lo0 = int.from_bytes(L0[on][:4].tobytes(), "little")
            lo1 = int.from_bytes(L1[on][:4].tobytes(), "little")
            assert (lo0 - lo1) % 2**32 == beta % 2**32


def test_walkthrough_L4(O):
    """Paper's L = 4 example: Eval(k, 3) = P(2, 3) needs P(1, 1), which needs P(0, 0).
    The leaf seeds at depth 2 must be the children of the depth-1 seeds
    with index j // 2, child j % 2."""
    k0, _ = O.gen(2, 3, 1, seed_for(4))
    root = k0[16:32]
    lvl1 = O.eval_level(k0, 1)
    lvl2 = O.eval_level(k0, 2)

    def cw(t, c, d):
        off = 32 + 64 * (d - 1) + 32 * t + 16 * c
        return np.frombuffer(k0[off:off + 16].tobytes(), np.uint8)

    for j in range(2):
        p = np.frombuffer(O.prf(root.tobytes(), j), np.uint8)
        assert (lvl1[j] == (p ^ cw(tbit(root), j, 1))).all()
    for j in range(4):
        parent = lvl1[j // 2]
        p = np.frombuffer(O.prf(parent.tobytes(), j % 2), np.uint8)
        assert (lvl2[j] == (p ^ cw(tbit(parent), j % 2, 2))).all()
    leaf3 = int.from_bytes(lvl2[3][:4].tobytes(), "little")
    assert O.eval_point(k0, 3) == leaf3  # party 0 share is +low32


def test_work_counts(O):
    """Full evaluation makes exactly 2(L-1) PRF calls (one per child, L-1
    internal nodes, section 3.1); point evaluation n; Gen 4n PRF calls
    (O(log L)) and 3n+1 random draws."""
    for n in (1, 5, 11):
        O.reset_counts()
        k0, k1 = O.gen(n, 1, 1, seed_for(n))
        assert O.counts() == (4 * n, 3 * n + 1)
        O.reset_counts()
        O.eval_full(k0)
        assert O.counts() == (2 * ((1 << n) - 1), 0)
        O.reset_counts()
        O.eval_point(k1, (1 << n) - 1)
        assert O.counts() == (n, 0)


def test_key_sizes_match_table4(O):
    g = read_golden("paper_key_sizes.txt")
    for n, paper_bytes in g.items():
        n = int(n)
        # codeword payload = 4 codewords x 16 bytes per level
        assert O.key_size(n) - 32 == int(paper_bytes)
    assert O.key_size(20) - 32 == 1280  # "1.25 KB" at one million entries


def test_keys_share_codewords(O):
    k0, k1 = O.gen(12, 1000, 1, seed_for(12))
    assert k0[0] == 1 and k1[0] == 1 and k0[1] == 0 and k1[1] == 1
    assert k0[2] == 12 and k1[2] == 12
    assert (k0[32:] == k1[32:]).all()
    assert tbit(k0[16:32]) != tbit(k1[16:32])
    # determinism and seed dependence
    assert (O.gen(12, 1000, 1, seed_for(12))[0] == k0).all()
    assert not (O.gen(12, 1000, 1, seed_for(13))[0] == k0).all()


def test_gen_rejects_bad_arguments(O):
    with pytest.raises(ValueError):
        O.gen(0, 0, 1, bytes(16))
    with pytest.raises(ValueError):
        O.gen(33, 0, 1, bytes(16))
    with pytest.raises(ValueError):
        O.gen(5, 32, 1, bytes(16))


def numpy_answer(shares, table):
    """Independent product: uint64 with a mask after every product."""
    rows = table.shape[0]
    y = shares[:rows].astype(np.uint64)
    acc = np.zeros(table.shape[1], np.uint64)
    for j in range(rows):
        acc = (acc + ((y[j] * table[j].astype(np.uint64)) & 0xFFFFFFFF)) & 0xFFFFFFFF
    return acc.astype(np.uint32)


@pytest.mark.parametrize("rows,dim", [(50, 7), (64, 16), (1, 3), (33, 1), (200, 64)])
def test_answer_and_reconstruct(O, rows, dim):
    n = max(1, (rows - 1).bit_length())
    rng = np.random.default_rng([rows, dim])
    T = rng.integers(0, 2**32, (rows, dim), dtype=np.uint64).astype(np.uint32)
    for alpha in sorted({0, rows - 1, int(rng.integers(0, rows))}):
        for beta in (1, 2**32 - 1, 12345):
            k0, k1 = O.gen(n, alpha, beta, seed_for(rows, dim, alpha, beta))
            a0, a1 = O.answer(k0, T), O.answer(k1, T)
            assert (a0 == numpy_answer(O.eval_full(k0), T)).all()
            assert (a1 == numpy_answer(O.eval_full(k1), T)).all()
            want = ((T[alpha].astype(np.uint64) * beta) & 0xFFFFFFFF).astype(np.uint32)
            assert (O.reconstruct(a0, a1) == want).all()


def test_reconstruct_every_alpha_small_table(O):
    rng = np.random.default_rng(3)
    T = rng.integers(0, 2**32, (24, 5), dtype=np.uint64).astype(np.uint32)
    for alpha in range(24):
        k0, k1 = O.gen(5, alpha, 1, seed_for(24, alpha))
        assert (O.reconstruct(O.answer(k0, T), O.answer(k1, T)) == T[alpha]).all()


def test_answer_batch_matches_single(O):
    rng = np.random.default_rng(8)
    n, rows, dim = 9, 400, 12
    T = rng.integers(0, 2**32, (rows, dim), dtype=np.uint64).astype(np.uint32)
    alphas = rng.integers(0, rows, 10)
    seeds = [seed_for(8, q) for q in range(10)]
    K0, K1 = O.gen_batch(n, alphas, seeds)
    keys = np.concatenate([K0, K1])
    got = O.answer_batch(keys, T, nthreads=4)
    for q in range(20):
        assert (got[q] == O.answer(keys[q], T)).all()
    for q in range(10):
        assert (O.reconstruct(got[q], got[10 + q]) == T[alphas[q]]).all()


def test_answer_rejects_bad_shapes(O):
    k0, _ = O.gen(4, 3, 1, bytes(16))
    with pytest.raises(ValueError):
        O.answer(k0, np.zeros((17, 2), np.uint32))  # more rows than 2^n
    bad = k0.copy()
    bad[0] = 2  # unknown key version
    with pytest.raises(ValueError):
        O.answer(bad, np.zeros((16, 2), np.uint32))


@pytest.mark.parametrize("n,shards,dim", [(6, 2, 3), (9, 8, 5), (11, 4, 16), (8, 64, 2)])
def test_answer_slices_sum_to_the_answer(O, n, shards, dim):
    """Row sharding (section 3.2.7): the slices' answers, each by point
    evaluation, equal an independent numpy product over the full evaluation
    and sum to the whole table's answer mod 2^32; the two servers' slice
    answers reconstruct T[alpha] in the slice holding alpha and zero in every
    other slice."""
    rows = 1 << n
    size = rows // shards
    rng = np.random.default_rng([n, shards, dim])
    T = rng.integers(0, 2**32, (rows, dim), dtype=np.uint64).astype(np.uint32)
    alpha = int(rng.integers(0, rows))
    k0, k1 = O.gen(n, alpha, 1, seed_for(n, shards, dim))
    y0 = O.eval_full(k0)
    total = np.zeros(dim, np.uint64)
    for s in range(shards):
        r0 = s * size
        a0 = O.answer_slice(k0, T[r0:r0 + size], r0)
        a1 = O.answer_slice(k1, T[r0:r0 + size], r0)
        assert (a0 == numpy_answer(y0[r0:r0 + size], T[r0:r0 + size])).all()
        want = T[alpha] if r0 <= alpha < r0 + size else np.zeros(dim, np.uint32)
        assert (O.reconstruct(a0, a1) == want).all(), s
        total = (total + a0) & 0xFFFFFFFF
    assert (total.astype(np.uint32) == O.answer(k0, T)).all()


def test_answer_slice_ragged_and_rejects(O):
    """An unaligned, ragged slice still follows the definition; a slice past
    the domain is refused."""
    n, dim = 7, 4
    rng = np.random.default_rng(71)
    T = rng.integers(0, 2**32, (1 << n, dim), dtype=np.uint64).astype(np.uint32)
    k0, _ = O.gen(n, 100, 1, seed_for(71))
    y = O.eval_full(k0)
    for r0, cnt in ((0, 1), (5, 17), (100, 28), (127, 1)):
        got = O.answer_slice(k0, T[r0:r0 + cnt], r0)
        assert (got == numpy_answer(y[r0:r0 + cnt], T[r0:r0 + cnt])).all(), (r0, cnt)
    with pytest.raises(ValueError):
        O.answer_slice(k0, T[:2], 127)  # indices 127, 128: past 2^7
