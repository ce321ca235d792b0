"""The batched form (GPU, through the C ABI): ldc_build (LNOs, solve and density in one call,
no host wait before the end), its HIP-graph capture and replays, size buckets with launch grids
picked by ldc_tune and read back from the tuning cache.  Every result is compared with the
separate-call build bit for bit (same kernels in the same order) and with the oracle at the
parity bar (Sec. II.C (i)-(v))."""
import json

import numpy as np
import pytest

import oracle
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _rule(s, fixed=None):
    return dict(lambda_th=s["lambda_th"], k_min=s["k_min"], k_max=s["k_max"], fixed_rank=fixed)


def _separate(ldc, s, H, S, dprev, stream, fixed=None):
    import torch
    plan = ldc.Plan.from_system(s, stream=stream)
    D = torch.zeros_like(S)
    plan.lno(S, dprev, want_ranks=False, **_rule(s, fixed))
    plan.solve(H, S)
    mu, eb, ne = plan.density(s["n_electrons"], s["kT"], D)
    torch.cuda.synchronize()
    plan.close()
    return D.cpu().numpy(), mu, eb


@pytest.mark.parametrize("name", ["sc27", "fcc_slab"])
def test_build_and_graph_replays_match_separate_calls(small_systems, name):
    import torch
    import paper_1809_05637_amd as ldc
    s = small_systems(name)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        H, S = to_dev(s["H"]), to_dev(s["S"])
        D0 = torch.zeros_like(S)
        base = ldc.Plan.from_system(s, stream=stream)
        base.lno(S, None)
        base.solve(H, S)
        base.density(s["n_electrons"], s["kT"], D0)
        torch.cuda.synchronize()
        base.close()
        dprev = D0 if s["lno"] else None
        ref_D, ref_mu, ref_eb = _separate(ldc, s, H, S, dprev, stream)
        plan = ldc.Plan.from_system(s, stream=stream, use_graph=True)
        D = torch.zeros_like(S)
        for rep in range(4):
            print(f"[batched] {name} graph build {rep}", flush=True)
            mu, eb, ne = plan.build(H, S, dprev, s["n_electrons"], s["kT"], D, **_rule(s))
            torch.cuda.synchronize()
            got = D.cpu().numpy()
            assert np.array_equal(got, ref_D), rep
            assert mu == ref_mu and eb == ref_eb
            # eager work on the same stream between replays
            D.fill_(7.0)
            x = (S * 2.0).sum()
            torch.cuda.synchronize()
            del x
        inf = plan.info()
        assert inf["graph_captures"] == 1 and inf["graph_replays"] == 4
        # another output buffer: a new capture
        D2 = torch.zeros_like(S)
        plan.build(H, S, dprev, s["n_electrons"], s["kT"], D2, **_rule(s))
        torch.cuda.synchronize()
        assert np.array_equal(D2.cpu().numpy(), ref_D)
        assert plan.info()["graph_captures"] == 2
        plan.close()


def test_graph_replay_takes_new_fixed_ranks(small_systems):
    """The captured copy reads the fixed ranks from the staging buffer at every replay."""
    import torch
    import paper_1809_05637_amd as ldc
    s = small_systems("fcc_slab")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        H, S = to_dev(s["H"]), to_dev(s["S"])
        D0 = torch.zeros_like(S)
        plan = ldc.Plan.from_system(s, stream=stream, use_graph=True)
        plan.build(H, S, None, s["n_electrons"], s["kT"], D0)
        D = torch.zeros_like(S)
        for k in (2, 3, 2):
            fixed = np.full(s["n_atoms"], k, np.int32)
            plan.build(H, S, D0, s["n_electrons"], s["kT"], D, **_rule(s, fixed))
            torch.cuda.synchronize()
            ref_D, _, _ = _separate(ldc, s, H, S, D0, stream, fixed)
            assert np.array_equal(D.cpu().numpy(), ref_D), k
        assert plan.info()["graph_captures"] == 2  # plain DC and the fixed-rank build
        plan.close()


def test_tuned_buckets_and_cache(small_systems, tmp_path):
    import torch
    import paper_1809_05637_amd as ldc
    s = small_systems("fcc_slab")
    cache = str(tmp_path / "tune.json")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        H, S = to_dev(s["H"]), to_dev(s["S"])
        D0, D = torch.zeros_like(S), torch.zeros_like(S)
        plan = ldc.Plan.from_system(s, stream=stream, batched=True, use_graph=True, tune_cache=cache,
                                    workgroups=8)
        plan.build(H, S, None, s["n_electrons"], s["kT"], D0)
        ms = plan.tune(H, S, D0, s["n_electrons"], s["kT"], D, **_rule(s))
        assert ms > 0.0
        b1 = plan.buckets()
        assert plan.info()["tuned"] == 1 and sum(b["count"] for b in b1) == s["n_atoms"]
        mu, eb, ne = plan.build(H, S, D0, s["n_electrons"], s["kT"], D, **_rule(s))
        torch.cuda.synchronize()
        got = D.cpu().numpy()
        plan.close()
        entries = json.load(open(cache))["entries"]
        assert len(entries) == 1 and entries[0]["n_buckets"] == len(b1)
        # a new plan reads the launch choices back from the cache
        plan2 = ldc.Plan.from_system(s, stream=stream, batched=True, use_graph=True, tune_cache=cache,
                                     workgroups=8)
        plan2.build(H, S, None, s["n_electrons"], s["kT"], D0)
        plan2.build(H, S, D0, s["n_electrons"], s["kT"], D, **_rule(s))
        torch.cuda.synchronize()
        assert plan2.info()["tuned"] == 2 and plan2.buckets() == b1
        assert np.array_equal(D.cpu().numpy(), got)
        plan2.close()
    ref0 = oracle.density_build(s, dprev=None, workers=1)
    ref = oracle.density_build(s, dprev=ref0["D"], workers=1)
    err = float(np.abs(got - ref["D"]).max())
    print(f"[batched] tuned fcc_slab: max|dD|={err:.3e} dE/atom={abs(eb - ref['e_band']) / s['n_atoms']:.3e}",
          flush=True)
    assert err <= 1e-9 and abs(eb - ref["e_band"]) / s["n_atoms"] <= 1e-10
