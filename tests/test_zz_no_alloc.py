"""Calls for callers that cannot allocate: without a bound workspace every
answer call reports into the library's own per-device status array (a static
device array located once per device with hipGetSymbolAddress) and calls no
allocator.  Checked through the C ABI against the same calls with a
caller-bound workspace, on two calls in a row, the second smaller: outputs
bit-exact and equal to the oracle's, and each call's status its own."""
import numpy as np
import pytest

from conftest import cpu_threads
from paper_2301_10904_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pirmod(gpu_lib):
    from paper_2301_10904_amd import pir

    pir.set_workspace(None)
    yield pir
    pir.set_workspace(None)


@pytest.mark.parametrize("prf", [0, 1])
def test_library_workspace_matches_a_bound_one(O, pirmod, prf):
    import torch

    ws = pirmod.workspace()
    calls = [(1 << 14, 64, 40), (3000, 16, 5)]  # the second call smaller
    for i, (rows, dim, nkeys) in enumerate(calls):
        seed = 80 + 10 * i + prf
        n = max(1, (rows - 1).bit_length())
        T = W.make_table(rows, dim, seed)
        a = W.uniform_indices(rows, nkeys, seed)
        K0, _ = O.gen_batch(n, a, W.key_seeds(nkeys, seed), prf_id=prf)
        bad = K0.copy()
        bad[nkeys - 1, 1] = 5  # the last key's party is out of range
        Td = T.cuda()
        want = O.answer_batch(K0, T.numpy().view(np.uint32), nthreads=cpu_threads())
        for keys, status in ((K0, pirmod.PIR_OK), (bad, pirmod.PIR_EKEY)):
            kd = torch.from_numpy(keys).cuda()
            pirmod.set_workspace(None)
            lib_out = pirmod.answer(kd, Td, prf=prf)
            torch.cuda.synchronize()
            assert pirmod.check_status() == status, (i, status)
            pirmod.set_workspace(ws)
            try:
                ws_out = pirmod.answer(kd, Td, prf=prf)
                assert pirmod.workspace_status(ws) == status
            finally:
                pirmod.set_workspace(None)
            torch.cuda.synchronize()
            g_lib = lib_out.cpu().numpy().view(np.uint32)
            g_ws = ws_out.cpu().numpy().view(np.uint32)
            assert (g_lib == g_ws).all(), i
            if status == pirmod.PIR_OK:
                assert (g_lib == want).all(), i
            else:
                assert (g_lib[-1] == 0).all() and (g_lib[:-1] == want[:-1]).all(), i
