"""Per-call status in a caller's workspace (include/pir.h: pir_set_workspace,
pir_workspace_status), on the GPU.

Each answer call clears its status word with its first kernel and sets
PIR_STATUS_BAD_KEY there for a key with a bad header; the word is the one of
the workspace bound by the calling thread.  Two streams with a workspace
each report independently; a call that is split over several launches (a
remainder past whole groups of 16 keys, several tables) reports once; a
captured graph reports the status of each replay.  Outputs are checked
against the oracle as everywhere else.
"""
import numpy as np
import pytest

from conftest import cpu_threads
from paper_2301_10904_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pirmod(gpu_lib):
    from paper_2301_10904_amd import pir

    yield pir
    pir.set_workspace(None)


def keyset(O, rows, count, seed, prf=0):
    n = max(1, (rows - 1).bit_length())
    a = W.uniform_indices(rows, count, seed)
    K0, _ = O.gen_batch(n, a, W.key_seeds(count, seed), prf_id=prf)
    return K0


def test_two_streams_each_with_its_own_workspace(O, pirmod):
    import torch

    rows, dim = 1 << 12, 64
    T = W.make_table(rows, dim, 31)
    Tn, Td = T.numpy().view(np.uint32), T.cuda()
    good = keyset(O, rows, 40, 31)
    bad = good.copy()
    bad[7, 1] = 2  # party 2 does not exist
    want = O.answer_batch(good, Tn, nthreads=cpu_threads())
    streams = (torch.cuda.Stream(), torch.cuda.Stream())
    spaces = (pirmod.workspace(), pirmod.workspace())
    kd = {"good": torch.from_numpy(good).cuda(), "bad": torch.from_numpy(bad).cuda()}
    torch.cuda.synchronize()
    for which in (("good", "bad"), ("bad", "good"), ("bad", "bad"), ("good", "good")):
        outs = []
        for st, ws, w in zip(streams, spaces, which):
            with torch.cuda.stream(st):
                pirmod.set_workspace(ws)
                outs.append(pirmod.answer(kd[w], Td, prf=0))
        pirmod.set_workspace(None)
        for st, ws, w in zip(streams, spaces, which):
            assert pirmod.workspace_status(ws, st) == (pirmod.PIR_EKEY if w == "bad" else pirmod.PIR_OK), which
        torch.cuda.synchronize()
        for o, w in zip(outs, which):
            g = o.cpu().numpy().view(np.uint32)
            if w == "good":
                assert (g == want).all()
            else:
                assert (g[7] == 0).all() and (np.delete(g, 7, 0) == np.delete(want, 7, 0)).all()


def test_each_call_reports_its_own_status(O, pirmod):
    """A call after a bad one starts from a clear word; the library's own
    workspace is untouched by calls that use a bound one."""
    import torch

    rows, dim = 3000, 16
    Td = W.make_table(rows, dim, 32).cuda()
    good = keyset(O, rows, 5, 32)
    bad = good.copy()
    bad[0, 3] = 9  # unknown PRF id
    ws = pirmod.workspace()
    pirmod.set_workspace(ws)
    try:
        pirmod.answer(torch.from_numpy(bad).cuda(), Td)
        assert pirmod.workspace_status(ws) == pirmod.PIR_EKEY
        pirmod.answer(torch.from_numpy(good).cuda(), Td)
        assert pirmod.workspace_status(ws) == pirmod.PIR_OK
        pirmod.answer(torch.from_numpy(bad).cuda(), Td)
    finally:
        pirmod.set_workspace(None)
    pirmod.answer(torch.from_numpy(good).cuda(), Td)
    torch.cuda.synchronize()
    assert pirmod.check_status() == pirmod.PIR_OK        # the library's own word
    assert pirmod.workspace_status(ws) == pirmod.PIR_EKEY  # the bound one kept its last call's status


@pytest.mark.parametrize("where", ["head", "tail"])
def test_a_split_call_reports_once(O, pirmod, where):
    """17 keys on 2^20 rows run as a launch over 16 keys and a second launch
    over the last one (pir_plan tail_keys = 1); a bad key in either launch is
    reported, because only the call's first launch clears the word."""
    import torch

    rows, dim = 1 << 20, 16
    assert pirmod.plan(17, rows, dim)["tail_keys"] == 1
    Td = W.make_table(rows, dim, 33, device="cuda")
    keys = keyset(O, rows, 17, 33)
    keys[3 if where == "head" else 16, 0] = 2  # bad version
    ws = pirmod.workspace()
    pirmod.set_workspace(ws)
    try:
        out = pirmod.answer(torch.from_numpy(keys).cuda(), Td)
        assert pirmod.workspace_status(ws) == pirmod.PIR_EKEY
    finally:
        pirmod.set_workspace(None)
    got = out.cpu().numpy().view(np.uint32)
    bad = 3 if where == "head" else 16
    assert (got[bad] == 0).all()
    other = (bad + 1) % 17
    assert (got[other] == O.answer(keys[other], Td.cpu().numpy().view(np.uint32))).all()


def test_status_of_each_graph_replay(O, pirmod):
    import torch

    rows, dim = 5000, 32
    T = W.make_table(rows, dim, 34)
    Tn, Td = T.numpy().view(np.uint32), T.cuda()
    good = keyset(O, rows, 20, 34)
    bad = good.copy()
    bad[19, 2] = 12  # wrong domain
    keys = torch.from_numpy(good).cuda()
    out = torch.empty((20, dim), dtype=torch.int32, device="cuda")
    ws = pirmod.workspace()
    pirmod.set_workspace(ws)
    try:
        pirmod.answer(keys, Td, out)  # eager, before capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            pirmod.answer(keys, Td, out)
    finally:
        pirmod.set_workspace(None)
    torch.cuda.synchronize()
    want = O.answer_batch(good, Tn, nthreads=cpu_threads())
    for rep, ks in enumerate([bad, good, bad, bad, good]):
        keys.copy_(torch.from_numpy(ks).cuda())
        g.replay()
        torch.cuda.synchronize()
        st = pirmod.workspace_status(ws)
        assert st == (pirmod.PIR_EKEY if ks is bad else pirmod.PIR_OK), rep
        got = out.cpu().numpy().view(np.uint32)
        if ks is bad:
            assert (got[19] == 0).all() and (got[:19] == want[:19]).all()
        else:
            assert (got == want).all()


def test_multi_table_call_reports_once(O, pirmod):
    import torch

    specs = [(1 << 12, 32, 40), (1 << 10, 32, 3), (5000, 64, 20)]
    tabs, keysets = [], []
    for i, (rows, dim, cnt) in enumerate(specs):
        tabs.append(W.make_table(rows, dim, 40 + i).cuda())
        keysets.append(keyset(O, rows, cnt, 40 + i))
    stride = max(k.shape[1] for k in keysets)
    keys = np.concatenate([np.pad(k, ((0, 0), (0, stride - k.shape[1]))) for k in keysets])
    ws = pirmod.workspace()
    pirmod.set_workspace(ws)
    try:
        for bad_at in (None, 0, 41, 60):
            ks = keys.copy()
            if bad_at is not None:
                ks[bad_at, 0] = 3
            pirmod.answer_multi(tabs, [s[2] for s in specs], torch.from_numpy(ks).cuda())
            want = pirmod.PIR_OK if bad_at is None else pirmod.PIR_EKEY
            assert pirmod.workspace_status(ws) == want, bad_at
    finally:
        pirmod.set_workspace(None)


def test_a_not_ready_query_before_a_call_is_not_an_error(O, pirmod):
    """An event query that finds its event not reached leaves "not ready" as
    the thread's last runtime error; the next library call must not mistake
    it for a failure of its own launches."""
    import torch

    rows, dim = 1 << 16, 64
    T = W.make_table(rows, dim, 35)
    Td = T.cuda()
    big = torch.from_numpy(keyset(O, rows, 512, 35)).cuda()
    small = keyset(O, rows, 3, 36)
    torch.cuda.synchronize()
    seen_not_ready = False
    for _ in range(3):
        pirmod.answer(big, Td)  # a few ms of work
        ev = torch.cuda.Event()
        ev.record()
        seen_not_ready |= not ev.query()
        got = pirmod.answer(torch.from_numpy(small).cuda(), Td)  # raises on a launch error
        torch.cuda.synchronize()
        want = O.answer_batch(small, T.numpy().view(np.uint32), nthreads=cpu_threads())
        assert (got.cpu().numpy().view(np.uint32) == want).all()
    assert seen_not_ready


@pytest.mark.parametrize("bound", [False, True])
@pytest.mark.parametrize("prf", [0, 1])
def test_one_launch_calls_leave_the_workspace_clean(O, pirmod, bound, prf):
    """A run of calls of one or two keys (the single-query path), a bad key
    among them and a larger call in between, on the library's own workspace
    or a bound one: each answers as the oracle and reports its own status."""
    import torch

    shapes = [(1 << 14, 64), (3000, 16), (1 << 16, 100)]
    ws = pirmod.workspace() if bound else None
    pirmod.set_workspace(ws)
    try:
        for i, (rows, dim) in enumerate(shapes):
            seed = 200 + 10 * i + prf
            n = max(1, (rows - 1).bit_length())
            T = W.make_table(rows, dim, seed)
            Tn, Td = T.numpy().view(np.uint32), T.cuda()
            a = W.uniform_indices(rows, 20, seed)
            K, _ = O.gen_batch(n, a, W.key_seeds(20, seed), prf_id=prf)
            want = O.answer_batch(K, Tn, nthreads=cpu_threads())
            bad = K[:2].copy()
            bad[1, 0] = 9  # bad version on the second key
            for keys, idx, st in ((K[:1], [0], 0), (K[:2], [0, 1], 0), (bad, [0], 1), (K[1:2], [1], 0),
                                  (K, list(range(20)), 0), (K[:1], [0], 0)):
                assert pirmod.plan(len(keys), rows, dim, prf=prf)["workgroups"] > 1
                out = pirmod.answer(torch.from_numpy(np.ascontiguousarray(keys)).cuda(), Td, prf=prf)
                torch.cuda.synchronize()
                got = out.cpu().numpy().view(np.uint32)
                status = pirmod.workspace_status(ws) if bound else pirmod.check_status()
                assert status == (pirmod.PIR_EKEY if st else pirmod.PIR_OK), (i, len(keys), st)
                if st:
                    assert (got[0] == want[0]).all() and (got[1] == 0).all()
                else:
                    assert (got == want[idx]).all(), (i, len(keys))
    finally:
        pirmod.set_workspace(None)


def test_one_key_call_replays_in_a_graph(O, pirmod):
    """A captured one-key call replayed with new keys, with eager calls on the
    library's own workspace in between: every replay answers as the oracle
    and reports its status in the bound workspace."""
    import torch

    rows, dim = 1 << 15, 64
    T = W.make_table(rows, dim, 37)
    Tn, Td = T.numpy().view(np.uint32), T.cuda()
    sets = [keyset(O, rows, 1, 300 + i) for i in range(3)]
    bad = sets[0].copy()
    bad[0, 2] = 3
    keys = torch.from_numpy(sets[0]).cuda()
    out = torch.empty((1, dim), dtype=torch.int32, device="cuda")
    ws = pirmod.workspace()
    pirmod.set_workspace(ws)
    try:
        pirmod.answer(keys, Td, out)  # eager, before capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            pirmod.answer(keys, Td, out)
    finally:
        pirmod.set_workspace(None)
    torch.cuda.synchronize()
    for rep, ks in enumerate([sets[1], bad, sets[2], sets[0], bad, sets[1]]):
        keys.copy_(torch.from_numpy(ks).cuda())
        out.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint32)
        if ks is bad:
            assert pirmod.workspace_status(ws) == pirmod.PIR_EKEY and (got == 0).all(), rep
        else:
            assert pirmod.workspace_status(ws) == pirmod.PIR_OK, rep
            assert (got == O.answer_batch(ks, Tn, nthreads=cpu_threads())).all(), rep
        other = pirmod.answer(torch.from_numpy(sets[2]).cuda(), Td)  # eager work on the library's workspace
        torch.cuda.synchronize()
        assert (other.cpu().numpy().view(np.uint32) == O.answer_batch(sets[2], Tn, nthreads=cpu_threads())).all()


def test_a_stalled_wait_is_reported_and_the_kernel_ends(O, pirmod):
    """The stream kernel's bounded waits forced to give up from the host (a
    wait limit of one try): every wave leaves its loop, the kernel ends, and
    the call reports PIR_ESTALL, in a bound workspace and in the library's
    own; with the default limit restored the same keys answer exactly and
    report PIR_OK."""
    import torch

    rows, dim = 1 << 22, 64
    assert pirmod.plan(1, rows, dim)["kernel"] == pirmod.KERNEL_STREAM
    Td = W.make_table(rows, dim, 41, device="cuda")
    a = W.uniform_indices(rows, 1, 41)
    K0, K1 = O.gen_batch(22, a, W.key_seeds(1, 41), prf_id=0)
    k0, k1 = torch.from_numpy(K0).cuda(), torch.from_numpy(K1).cuda()
    ws = pirmod.workspace()
    try:
        pirmod.set_wait_limit(1)
        pirmod.set_workspace(ws)
        pirmod.answer(k0, Td)
        assert pirmod.workspace_status(ws) == pirmod.PIR_ESTALL
        pirmod.set_workspace(None)
        pirmod.answer(k1, Td)
        torch.cuda.synchronize()
        assert pirmod.check_status() == pirmod.PIR_ESTALL
    finally:
        pirmod.set_wait_limit(0)
        pirmod.set_workspace(None)
    pirmod.set_workspace(ws)
    try:
        o0 = pirmod.answer(k0, Td)
        assert pirmod.workspace_status(ws) == pirmod.PIR_OK
    finally:
        pirmod.set_workspace(None)
    o1 = pirmod.answer(k1, Td)
    torch.cuda.synchronize()
    assert pirmod.check_status() == pirmod.PIR_OK
    rec = pirmod.reconstruct(o0.cpu().numpy().view(np.uint32)[0], o1.cpu().numpy().view(np.uint32)[0])
    assert (rec == W.table_rows_np(a, dim, 41)[0]).all()



def test_a_stalled_pair_wait_ends_the_kernel(O, pirmod):
    """The wave pairs' bounded waits (rows of 65..128 words) with a wait limit
    of one try: the kernel ends whatever its waits see, and the call reports
    PIR_ESTALL, or PIR_OK with exact answers if no wait had to give up; with
    the default limit restored the same keys answer exactly and report PIR_OK."""
    import torch

    rows, dim, nk = 1 << 18, 128, 64
    assert pirmod.plan(nk, rows, dim)["kernel"] == pirmod.KERNEL_WAVES
    T = W.make_table(rows, dim, 43)
    Td = T.cuda()
    K = keyset(O, rows, nk, 43)
    want = O.answer_batch(K, T.numpy().view(np.uint32), nthreads=cpu_threads())
    keys = torch.from_numpy(K).cuda()
    try:
        pirmod.set_wait_limit(1)
        out = pirmod.answer(keys, Td)
        torch.cuda.synchronize()
        st = pirmod.check_status()
        assert st in (pirmod.PIR_ESTALL, pirmod.PIR_OK)
        if st == pirmod.PIR_OK:
            assert (out.cpu().numpy().view(np.uint32) == want).all()
    finally:
        pirmod.set_wait_limit(0)
    out = pirmod.answer(keys, Td)
    torch.cuda.synchronize()
    assert pirmod.check_status() == pirmod.PIR_OK
    assert (out.cpu().numpy().view(np.uint32) == want).all()
