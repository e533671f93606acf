"""The serving loop on the GPU: Poisson arrivals over several resident tables.

The run starts right after the tables are generated on the default stream, so
the server stream must wait for that work (a served answer computed on a
half-written table fails the reconstruction check).

Checks the bookkeeping (every offered request is completed or rejected,
latencies are positive), the HBM admission of tables, and the answers: for a
sample of served requests, the served share plus its partner's share
reconstructs T[alpha] (the partner is answered through pir_answer directly).
"""
import numpy as np
import pytest

from paper_2301_10904_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prf", ["aes128", "chacha20"])
def test_serve_poisson_four_tables(gpu_lib, prf):
    import torch

    from paper_2301_10904_amd import pir
    from paper_2301_10904_amd.serve import PirServer

    logs = [10, 12, 14, 20]
    total = sum((1 << lg) * 32 * 4 for lg in logs)  # a 128 MiB table among them
    srv = PirServer(hbm_budget_bytes=total, max_batch=256, max_queue=512, max_inflight=2, prf=prf)
    pool, alphas = [], []
    for i, lg in enumerate(logs):
        T = W.make_table(1 << lg, 32, 60 + i, device="cuda")
        assert srv.admit_table(T) == i
        a = W.uniform_indices(1 << lg, 64, 60 + i)
        K0, K1 = pir.gen_batch(lg, a, W.key_seeds(64, 60 + i), prf=prf)
        pool.append(np.concatenate([K0, K1]))
        alphas.append(np.concatenate([a, a]))
    # the budget is exhausted: one more table is refused
    assert srv.admit_table(W.make_table(16, 32, 1, device="cuda")) == -1
    stride = (max(k.shape[1] for k in pool) + 15) // 16 * 16
    pool = [np.pad(k, ((0, 0), (0, stride - k.shape[1]))) for k in pool]
    checked = []

    def check(t, ki, row):
        partner = ki + 64 if ki < 64 else ki - 64
        pk = torch.from_numpy(pool[t][partner:partner + 1]).cuda()
        other = pir.answer(pk, srv.tables[t][0], prf=prf).cpu().numpy().view(np.uint32)[0]
        want = W.table_rows_np([alphas[t][ki]], 32, 60 + t)[0]
        checked.append(bool((pir.reconstruct(row, other) == want).all()))

    n = 6000
    arr = W.poisson_arrivals(20000.0, n, 5)
    rng = np.random.default_rng(9)
    tids = rng.integers(0, 4, n)
    kidx = rng.integers(0, 128, n)
    st = srv.run(arr, tids, pool, kidx, stride, check=check)
    s = st.summary()
    assert s["completed"] + s["rejected"] == n
    assert s["completed"] > 0 and s["p50_ms"] > 0 and s["p99_ms"] >= s["p50_ms"]
    assert checked and all(checked), checked
