"""Many independent instances in one captured graph: every replay equals
eager single-instance steps bitwise, for instances of different lattices,
sample counts, architectures and forms (the BF16 split-form instances with
their Grams in one grouped launch)."""
import pytest
import torch

from tests.gpu_common import gpu, need_gpu

pytestmark = gpu


def _instances(pm, tag):
    specs = [
        (dict(Lx=12, Ly=1, dim=1, hidden=32, dtype="f64", seed=1), pm.hamiltonian("tfim", pbc=True), 96, 0),
        (dict(Lx=10, Ly=1, dim=1, hidden=16, complex_head=True, dtype="f64", seed=2),
         pm.hamiltonian("cluster"), 64, 0),
        (dict(Lx=4, Ly=3, dim=2, hidden=32, marshall=True, zero_mag=True, dtype="f32", seed=3),
         pm.hamiltonian("j1j2", J=1.0, J2=0.0), 130, 1),
        (dict(Lx=3, Ly=4, dim=2, hidden=64, complex_head=True, marshall=True, dtype="f32", seed=4),
         pm.hamiltonian("j1j2", J=1.0, J2=0.5), 70, 2),
        # two BF16 split-form instances: their Grams run in one grouped
        # launch (3 and 10 tile pairs, ragged last tiles)
        (dict(Lx=14, Ly=1, dim=1, hidden=32, dtype="f32", seed=5), pm.hamiltonian("tfim", pbc=True),
         200, 1),
        (dict(Lx=11, Ly=1, dim=1, hidden=16, complex_head=True, dtype="f32", seed=6),
         pm.hamiltonian("cluster"), 230, 1),
    ]
    out = []
    for k, (margs, ham, Ns, form) in enumerate(specs):
        m = pm.Model(max_Ns=Ns, **margs)
        out.append(dict(model=m, ham=ham, Ns=Ns, eta=0.05, lam=1e-2, mu=0.3, key=100 + k,
                        form=form))
    return out


def test_batch_graph_matches_eager():
    need_gpu()
    import paper_2608_18065_amd as pm
    batched = _instances(pm, "b")
    eager = _instances(pm, "e")
    b = pm.Batch(batched)
    moms = [torch.zeros(i["model"].Np, dtype=torch.float64, device="cuda") for i in eager]
    for step in range(3):
        b.step()
        torch.cuda.synchronize()
        junk = torch.randn(4096, device="cuda").sum()   # eager work between replays
        for k, inst in enumerate(eager):
            o = inst["model"].step(inst["ham"], inst["Ns"], inst["eta"], inst["lam"], inst["mu"],
                                   moms[k], inst["key"], step, form=inst["form"])
            torch.cuda.synchronize()
            ob = b.outputs[k]
            assert int(b.counters[k].item()) == step + 1
            for key in ("energy", "dtheta", "status", "eloc", "sigma"):
                assert torch.equal(o[key], ob[key]), (step, k, key)
            assert torch.equal(moms[k], b.momentum[k]), (step, k)
            assert torch.equal(inst["model"].get_params(), batched[k]["model"].get_params())
        del junk
    b.close()


def test_tunables_roundtrip_and_effect_free():
    need_gpu()
    import paper_2608_18065_amd as pm
    m1 = pm.Model(16, hidden=64, dtype="f32", seed=9, max_Ns=256)
    m2 = pm.Model(16, hidden=64, dtype="f32", seed=9, max_Ns=256)
    m2.set_tunable("gram_split", 3)
    m2.set_tunable("eloc_grid", 7)
    m2.set_tunable("sample_r", 4)
    m2.set_tunable("jac_parts", 4)
    assert m2.get_tunable("gram_split") == 3
    with pytest.raises(pm.MinsrError):
        m2.set_tunable("nonsense", 1)
    ham = pm.hamiltonian("tfim", pbc=True)
    outs, grams = [], []
    for m in (m1, m2):
        mom = torch.zeros(m.Np, dtype=torch.float64, device="cuda")
        outs.append(m.step(ham, 256, 0.1, 1e-3, 0.0, mom, 5, 0, form=pm.FORM_FP32_PLAIN))
        grams.append(m.intermediates(pm.FORM_FP32_PLAIN)["T"].double())
    torch.cuda.synchronize()
    # split-K partial sums of T are FP32 over different chunkings
    scale = float(grams[0].abs().max())
    assert float((grams[0] - grams[1]).abs().max()) < 1e-5 * scale
    # launch parameters change scheduling, not the samples or local energies
    assert torch.equal(outs[0]["sigma"], outs[1]["sigma"])
    assert torch.equal(outs[0]["eloc"], outs[1]["eloc"])
    # the Gram split changes only the FP32 summation order of T's partial
    # sums; the solve amplifies that by up to cond(T + lambda I), so the
    # directions are held to the same 2e-2 relative bound as the
    # low-precision forms against the FP64 reference
    d0, d1 = outs[0]["dtheta"], outs[1]["dtheta"]
    assert float((d0 - d1).norm() / d0.norm()) < 2e-2


def test_autotuner_picks_and_caches(tmp_path):
    need_gpu()
    import paper_2608_18065_amd as pm
    from paper_2608_18065_amd import autotune
    m = pm.Model(16, hidden=64, dtype="f32", seed=4, max_Ns=256)
    ham = pm.hamiltonian("tfim", pbc=True)
    cache = str(tmp_path / "tune.json")
    res = autotune.tune(m, ham, 256, reps=2, cache=cache)
    assert set(res) == set(autotune.CANDIDATES)
    for key, (best, times) in res.items():
        assert best in autotune.CANDIDATES[key]
        assert times[best] == min(times.values())
        assert m.get_tunable(key) == best
    # a fresh model of the same shape picks the cached values up
    m2 = pm.Model(16, hidden=64, dtype="f32", seed=5, max_Ns=256)
    applied = autotune.apply(m2, 256, cache=cache)
    assert applied == {k: v[0] for k, v in res.items()}
    for k, v in applied.items():
        assert m2.get_tunable(k) == v
