"""The library's calls inside a captured HIP graph (torch.cuda.CUDAGraph).

A caller may capture pir_answer / pir_answer_bins: they enqueue only kernels
(the output is cleared by a fill kernel, not a memset node).  Each graph is
replayed several times with eager work between the replays (new keys copied
into the captured input, other library calls, synchronisations), and every
replay is checked against the oracle on the keys it saw.
"""
import numpy as np
import pytest

from conftest import cpu_threads
from paper_2301_10904_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pirmod(gpu_lib):
    from paper_2301_10904_amd import pir

    return pir


@pytest.mark.parametrize("pairs,prf", [(40, 0), (3, 1)])  # wave kernel with AES, small-batch kernel with ChaCha20
def test_answer_replays_in_a_graph(O, pirmod, pairs, prf):
    import torch

    rows, dim, n, seed = 5000, 64, 13, 90 + prf
    T = W.make_table(rows, dim, seed)
    Tn = T.numpy().view(np.uint32)
    Td = T.cuda()
    sets = []
    for s in range(3):
        a = W.uniform_indices(rows, pairs, seed * 10 + s)
        K0, K1 = O.gen_batch(n, a, W.key_seeds(pairs, seed * 10 + s), prf_id=prf)
        sets.append(np.concatenate([K0, K1]))
    keys = torch.from_numpy(sets[0]).cuda()
    out = torch.empty((2 * pairs, dim), dtype=torch.int32, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pirmod.answer(keys, Td, out, prf=prf)  # eager call before capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pirmod.answer(keys, Td, out, prf=prf)
    torch.cuda.synchronize()
    for rep in range(6):
        ks = sets[rep % 3]
        keys.copy_(torch.from_numpy(ks).cuda())
        out.fill_(-1)  # a replay must overwrite every word
        g.replay()
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint32)
        assert (got == O.answer_batch(ks, Tn, nthreads=cpu_threads())).all(), rep
        # eager library work between replays, on another output
        other = pirmod.answer(keys[:2].contiguous(), Td, prf=prf)
        torch.cuda.synchronize()
        assert (other.cpu().numpy().view(np.uint32) == got[:2]).all()


def test_bins_replay_in_a_graph(O, pirmod):
    import torch

    rows, dim, bin_log, clients, seed = 3000, 32, 8, 18, 97
    T = W.make_table(rows, dim, seed)
    Tn = T.numpy().view(np.uint32)
    Td = T.cuda()
    nb = -(-rows // (1 << bin_log))
    sets = []
    for s in range(2):
        rng = np.random.default_rng([seed, s])
        alphas = [int(rng.integers(0, min(1 << bin_log, rows - (c % nb) * (1 << bin_log))))
                  for c in range(clients * nb)]
        K0, _ = O.gen_batch(bin_log, alphas, W.key_seeds(len(alphas), seed * 10 + s))
        sets.append(K0)
    keys = torch.from_numpy(sets[0]).cuda()
    out, views = pirmod.answer_bins([Td], [clients], [bin_log], keys)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pirmod.answer_bins([Td], [clients], [bin_log], keys, out=out)
    for rep in range(4):
        ks = sets[rep % 2]
        keys.copy_(torch.from_numpy(ks).cuda())
        out.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        got = views[0].cpu().numpy().view(np.uint32)
        assert (got == O.answer_bins(ks, Tn, bin_log, clients, nthreads=cpu_threads())).all(), rep
