"""GPU tests of multi-request batching and the serving loop: each request's
result is the same alone and in a mix (bit for bit by construction; asserted
against the alone run exactly and against the oracle at 1e-9)."""
import numpy as np
import pytest

import graphgen as gg
import paper_2401_02472_amd as bcm
from paper_2401_02472_amd.serving import BCServer
from tests.gpu_checks import check_bc, oracle_bc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    bcm.load_library()


def alone(G, src):
    import torch
    out = torch.empty(G.n, dtype=torch.float64, device="cuda")
    G.run_multi([src], [out])
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_run_multi_mix_equals_alone_bitwise():
    import torch
    g = gg.rmat(13, 16, seed=21)
    rng = np.random.default_rng(3)
    reqs = [gg.sample_sources(g, k, seed=30 + i) for i, k in
            enumerate([1, 8, 64, 3, 100, 8, 64, 1, 17, 130])]
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        outs = [torch.empty(g.n, dtype=torch.float64, device="cuda") for _ in reqs]
        order = rng.permutation(len(reqs))
        G.run_multi([reqs[i] for i in order], [outs[i] for i in order])
        torch.cuda.synchronize()
        for i, src in enumerate(reqs):
            got = outs[i].cpu().numpy()
            assert np.array_equal(got, alone(G, src)), f"request {i} differs in the mix"
            check_bc(got, oracle_bc(g, src))


def test_run_multi_empty_and_duplicates():
    import torch
    g = gg.rmat(10, 8, seed=5)
    with bcm.Graph(g.n, g.row_ptr, g.col_idx) as G:
        outs = [torch.full((g.n,), 7.0, dtype=torch.float64, device="cuda") for _ in range(3)]
        reqs = [np.zeros(0, np.int32), np.array([3, 3, 5], np.int32), np.array([9], np.int32)]
        G.run_multi(reqs, outs)
        torch.cuda.synchronize()
        assert np.all(outs[0].cpu().numpy() == 0)
        check_bc(outs[1].cpu().numpy(), oracle_bc(g, reqs[1]))
        check_bc(outs[2].cpu().numpy(), oracle_bc(g, reqs[2]))


def test_server_mix_equals_alone():
    graphs = {"s12": gg.rmat(12, 16, seed=1), "s13": gg.rmat(13, 16, seed=2),
              "grid": gg.grid_road(48, 48, seed=3)}
    Gs = {k: bcm.Graph(g.n, g.row_ptr, g.col_idx) for k, g in graphs.items()}
    try:
        srv = BCServer(Gs, budget=8 << 30, slots=3, max_lanes=256)
        rng = np.random.default_rng(7)
        sub = []
        for i in range(36):
            gid = list(graphs)[i % 3]
            k = int(rng.choice([1, 8, 64]))
            src = gg.sample_sources(graphs[gid], k, seed=100 + i)
            sub.append((gid, src, srv.submit(gid, src)))
        for gid, src, fut in sub:
            got = fut.result(timeout=120)
            want = alone(Gs[gid], src)
            assert np.array_equal(got, want)
            check_bc(got, oracle_bc(graphs[gid], src))
        srv.close()
        st = srv.latency_stats()
        assert st["requests"] == 36
        assert srv.launches < 36           # requests were packed together
    finally:
        for G in Gs.values():
            G.close()


def test_server_keeps_resident_pools_within_budget():
    """The library keeps each graph's workspaces pooled after a launch; the
    server counts them against its budget and frees idle graphs' pools (least
    recently used first) when a launch would not fit.  Device memory in use,
    measured after every launch, stays within the budget."""
    import threading

    import torch
    from paper_2401_02472_amd.serving import GpuExecutor

    specs = [(17, 1), (17, 2), (16, 3), (15, 4)]
    graphs = {f"s{sc}-{sd}": gg.rmat(sc, 16, seed=sd) for sc, sd in specs}
    Gs = {k: bcm.Graph(g.n, g.row_ptr, g.col_idx) for k, g in graphs.items()}
    try:
        opt = bcm.make_options(bcm.BC_MODE_BATCHED, concurrency=1)
        ws = {k: G.workspace_bytes(64, opt) for k, G in Gs.items()}
        # one launch on the largest graph fits; every graph's pool at once does not
        budget = int(1.6 * max(ws.values()))
        assert sum(ws.values()) > budget
        torch.cuda.synchronize()
        free, total = torch.cuda.mem_get_info()
        base = total - free
        peak = {"used": 0, "held": 0}
        lock = threading.Lock()

        class Watch(GpuExecutor):
            def run(self, slot, gid, reqs):
                out = super().run(slot, gid, reqs)
                f, t = torch.cuda.mem_get_info()
                held = sum(G.workspace_held() for G in Gs.values())
                with lock:
                    peak["used"] = max(peak["used"], t - f - base)
                    peak["held"] = max(peak["held"], held)
                return out

        srv = BCServer(Gs, budget=budget, slots=3, max_lanes=64, executor=Watch(Gs, 3))
        rng = np.random.default_rng(11)
        sub = []
        for i in range(40):
            gid = list(graphs)[int(rng.integers(len(graphs)))]
            k = int(rng.choice([1, 8, 64]))
            src = gg.sample_sources(graphs[gid], k, seed=500 + i)
            sub.append((gid, src, srv.submit(gid, src)))
        for gid, src, fut in sub:
            fut.result(timeout=120)
        srv.close()
        print(f"# budget {budget / 2**20:.0f} MiB, pools at most {peak['held'] / 2**20:.0f} MiB, "
              f"device memory at most {peak['used'] / 2**20:.0f} MiB above the start, "
              f"{srv.trims} pool trims", flush=True)
        assert srv.trims > 0
        assert peak["held"] <= budget
        # outputs are in the budget; torch may cache their blocks, and the
        # device allocator rounds allocations up
        assert peak["used"] <= budget + (64 << 20)
        for gid, src, fut in sub[:6]:
            check_bc(fut.result(), oracle_bc(graphs[gid], src))
    finally:
        for G in Gs.values():
            G.close()
