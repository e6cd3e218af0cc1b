"""Batched persistent apply == unbatched applies; tuning candidates agree;
batched PCG reaches the oracle's solutions."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch

import oracle
import workloads as W
from gpu_util import dev, host, rel, rel_max, say

pytestmark = pytest.mark.gpu

vpp = pytest.importorskip("paper_2401_07805_amd")


def test_batch_equals_single(tmp_path):
    wls = W.batch_meshes(sizes=(4, 6, 9, 5), nrhs=3)
    probs = []
    for wl in wls:
        p = vpp.Problem.from_mesh(wl.mesh)
        p.set_phi(dev(wl.phi))
        probs.append(p)
    cache = str(tmp_path / "tune.json")
    say("batch create")
    bt = vpp.Batch(probs, [3] * len(probs), tune_cache=cache)
    xs = [dev(wl.vectors[r]) for wl in wls for r in range(3)]
    ys = [torch.empty_like(x) for x in xs]
    say("batch apply", bt.config)
    bt.apply(xs, ys)
    i = 0
    for p, wl in zip(probs, wls):
        for r in range(3):
            y1 = host(p.apply(xs[i]))
            assert rel(host(ys[i]), y1) < 1e-14
            i += 1
    # replays of the graph give identical results
    y_before = [host(y).copy() for y in ys]
    for _ in range(3):
        bt.apply(xs, ys)
    for a, y in zip(y_before, ys):
        assert rel(host(y), a) < 1e-14
    # the tuning cache was written and is reused
    import json
    data = json.load(open(cache))
    assert len(data["entries"]) == 1
    bt2 = vpp.Batch(probs, [3] * len(probs), tune_cache=cache)
    assert bt2.config == bt.config


def test_tune_and_candidate_invariance(tmp_path):
    wl = W.small_droplet(n=12, k=2, seed=3)
    prob = vpp.Problem.from_mesh(wl.mesh)
    prob.set_phi(dev(wl.phi))
    x = dev(wl.vectors[0])
    ys = []
    for cfg in vpp.config_candidates(2):
        prob.set_config(cfg["variant"], cfg["tile"])
        ys.append(host(prob.apply(x)))
    for y in ys[1:]:
        assert rel(y, ys[0]) < 1e-13
    cache = str(tmp_path / "c.json")
    say("tune")
    c1 = prob.tune(cache)
    c2 = prob.tune(cache)
    assert c1 == c2


def _batch_systems(nrhs=2):
    """Four single-sphere meshes (density ratios 1e4, 1e2, 1e4, 1e4) with the
    manufactured sine load of the mesh's own sphere and the phi-free sine load."""
    wls = W.batch_meshes(sizes=(4, 6, 9, 5), nrhs=nrhs)
    probs, systems = [], []
    for wl in wls:
        m = wl.mesh
        p = vpp.Problem.from_mesh(m)
        p.set_phi(dev(wl.phi))
        probs.append(p)
        op = oracle.Operator(m, phi=wl.phi)
        loads = (oracle.manufactured_sine_rhs(m, wl.extra["radius"], m.eps), oracle.sine_load(m))
        for r in range(nrhs):
            systems.append((p, op, loads[r % 2]))
    return probs, systems


def test_batch_cg_fp64_matches_oracle():
    """All (mesh, rhs) systems in lockstep: each reaches the oracle's direct
    solution, its true residual (oracle CSR) is below rtol, and the iteration
    counts (14 to 32 here, so systems stop at different chunks) agree with the
    oracle's PCG and with a single solve of the same system."""
    probs, systems = _batch_systems()
    say("batch cg create")
    bt = vpp.Batch(probs, [2] * len(probs))
    bs = [dev(b) for _, _, b in systems]
    xs = [torch.zeros_like(b) for b in bs]
    say("batch cg fp64", bt.config)
    infos = bt.cg_solve(bs, xs, rtol=1e-10, check_every=4)
    for i, ((prob, op, b), inf) in enumerate(zip(systems, infos)):
        x = host(xs[i])
        pref = spla.spsolve(op.to_scipy().tocsc(), b)
        res = np.linalg.norm(b - op.matvec(x)) / np.linalg.norm(b)
        _, oinf = op.pcg(b, rtol=1e-10)
        _, sinf = prob.cg_solve(bs[i], rtol=1e-10)
        print(i, inf, "true res", res, "err", rel(x, pref), "oracle it", oinf["iterations"],
              "single it", sinf["iterations"])
        assert inf["status"] == 0
        assert res < 1e-10 * 1.01
        assert abs(inf["true_rel_residual"] - res) < 1e-3 * res + 1e-14
        assert rel(x, pref) < 1e-8
        assert abs(inf["iterations"] - oinf["iterations"]) <= 2
        assert abs(inf["iterations"] - sinf["iterations"]) <= 2
    # the chunk length of the graph does not change the arithmetic
    xs2 = [torch.zeros_like(b) for b in bs]
    infos2 = bt.cg_solve(bs, xs2, rtol=1e-10)
    for a, b_, ia, ib in zip(xs, xs2, infos, infos2):
        assert torch.equal(a, b_)
        assert ia["iterations"] == ib["iterations"]


def test_batch_cg_edge_cases():
    """Zero and NaN right-hand sides, iteration limits and warm starts inside
    one batch: each system ends with its own status, the others are unaffected."""
    probs, systems = _batch_systems()
    bt = vpp.Batch(probs, [2] * len(probs))
    bs = [dev(b) for _, _, b in systems]
    bs[1] = torch.zeros_like(bs[1])                 # converged before any iteration
    bs[4] = bs[4].clone()
    bs[4][len(bs[4]) // 2] = float("nan")            # breakdown
    xs = [torch.zeros_like(b) for b in bs]
    say("batch cg edge cases")
    infos = bt.cg_solve(bs, xs, rtol=1e-10, raise_on_failure=False)
    for i, inf in enumerate(infos):
        if i == 1:
            assert inf["status"] == 0 and inf["iterations"] == 0
            assert float(xs[i].abs().max()) == 0.0
        elif i == 4:
            assert inf["status"] == 6
        else:
            _, op, b = systems[i]
            res = np.linalg.norm(b - op.matvec(host(xs[i]))) / np.linalg.norm(b)
            assert inf["status"] == 0 and res < 1e-10 * 1.01
    with pytest.raises(vpp.VppError) as e:
        bt.cg_solve(bs, [torch.zeros_like(b) for b in bs], rtol=1e-10)
    assert e.value.status == 6
    # iteration limit: every live system stops after exactly max_iter iterations
    good = [dev(b) for _, _, b in systems]
    infos = bt.cg_solve(good, [torch.zeros_like(b) for b in good], rtol=1e-14, max_iter=3,
                        raise_on_failure=False)
    assert all(inf["status"] == 5 and inf["iterations"] == 3 for inf in infos)
    # warm start from the solutions: the rule is relative to the new initial
    # residual, so the systems iterate again and converge
    xs = [torch.zeros_like(b) for b in good]
    bt.cg_solve(good, xs, rtol=1e-6)
    infos = bt.cg_solve(good, xs, rtol=1e-6)
    assert all(inf["status"] == 0 and inf["iterations"] >= 1 for inf in infos)
    # mixed precision runs the systems one after another and reaches the FP64 criterion
    xm = [torch.zeros_like(b) for b in good]
    infos = bt.cg_solve(good, xm, rtol=1e-8, precision="mixed")
    for (_, op, b), x, inf in zip(systems, xm, infos):
        res = np.linalg.norm(b - op.matvec(host(x))) / np.linalg.norm(b)
        assert inf["status"] == 0 and res < 1e-8 * 1.01


def test_batch_cg_mesh_above_lockstep_size():
    """A system of a mesh with at least 2^20 unknowns is solved on its own with
    the single-problem solver (bit-identical to vpp_cg_solve), next to lockstep
    systems of a small mesh that still reach the oracle's solution."""
    small = W.batch_meshes(sizes=(6,), nrhs=2)[0]
    big = W.small_droplet(n=52, k=2, seed=5)
    assert big.mesh.ndofs >= 1 << 20
    probs = []
    for wl in (small, big):
        p = vpp.Problem.from_mesh(wl.mesh)
        p.set_phi(dev(wl.phi))
        probs.append(p)
    op = oracle.Operator(small.mesh, phi=small.phi)
    b_small = oracle.sine_load(small.mesh)
    b_big = dev(big.vectors[0])
    bs = [dev(b_small), dev(b_small * -2.0), b_big]
    bt = vpp.Batch(probs, [2, 1])
    xs = [torch.zeros_like(b) for b in bs]
    say("batch cg with a large mesh", big.mesh.ndofs)
    infos = bt.cg_solve(bs, xs, rtol=1e-8)
    x1, inf1 = probs[1].cg_solve(b_big, rtol=1e-8)
    assert infos[2]["status"] == 0 and infos[2]["iterations"] == inf1["iterations"]
    assert torch.equal(xs[2], x1)
    pref = spla.spsolve(op.to_scipy().tocsc(), b_small)
    for x, scale, inf in zip(xs[:2], (1.0, -2.0), infos[:2]):
        assert inf["status"] == 0
        assert rel(host(x), scale * pref) < 1e-6


@pytest.mark.timeout(600)
def test_c3_batch_apply_against_oracle():
    """The batched workload at its real sizes (8 meshes of 16..64 cells per side,
    Q2, one seeded sphere each, ratios from {1e2, 1e3, 1e4}, 4 seeded right-hand
    sides per mesh): every output of one persistent batched apply against the
    oracle, at 1e-12 relative - all rows on the 16^3 and 24^3 meshes (CSR SpMV),
    1500 seeded rows plus every 997th row on the larger ones (row by row)."""
    wls = W.batch_meshes()
    probs, xs = [], []
    for wl in wls:
        p = vpp.Problem.from_mesh(wl.mesh)
        p.set_phi(dev(wl.phi))
        probs.append(p)
        xs += [dev(v) for v in wl.vectors]
    ys = [torch.empty_like(x) for x in xs]
    say("c3 batch create")
    bt = vpp.Batch(probs, [len(wl.vectors) for wl in wls])
    say("c3 batch apply", bt.config)
    bt.apply(xs, ys)
    torch.cuda.synchronize()
    i = 0
    rng = np.random.default_rng(77)
    for wl in wls:
        m = wl.mesh
        full = m.ncells[0] <= 24
        op = oracle.Operator(m, phi=wl.phi) if full else None
        rows = None if full else np.unique(np.concatenate([rng.choice(m.ndofs, 1500, replace=False),
                                                            np.arange(0, m.ndofs, 997)]))
        for r in range(len(wl.vectors)):
            y = host(ys[i])
            x = wl.vectors[r]
            if full:
                yref = op.matvec(x)
                err, errm = rel(y, yref), rel_max(y, yref)
            else:
                yr = oracle.apply_rows(m, wl.phi, x, rows)
                err, errm = rel(y[rows], yr), rel_max(y[rows], yr)
            say("c3 mesh", m.ncells[0], "ratio", wl.extra["ratio"], "rhs", r, f"err {err:.2e} max {errm:.2e}")
            assert err < 1e-12 and errm < 1e-12
            i += 1


def test_batch_q3_apply_against_oracle():
    """Q3 batches (a work item per (mesh, tile, rhs), the coefficient recomputed
    per item): five meshes of 4..13 cells per side (ragged tiles in every
    direction), density ratios from {1e2, 1e3, 1e4}, three right-hand sides
    each; every output against the oracle's CSR product at 1e-12 and against
    the single-problem apply, for every batch kernel configuration of degree 3,
    and graph replays repeat the bits."""
    wls = W.batch_meshes(sizes=(4, 6, 9, 5, 13), nrhs=3, k=3)
    probs, ops = [], []
    for wl in wls:
        p = vpp.Problem.from_mesh(wl.mesh)
        p.set_phi(dev(wl.phi))
        probs.append(p)
        ops.append(oracle.Operator(wl.mesh, phi=wl.phi))
    xs = [dev(wl.vectors[r]) for wl in wls for r in range(3)]
    say("q3 batch create")
    bt = vpp.Batch(probs, [3] * len(probs))
    assert bt.config["variant"] == 4
    ys = [torch.empty_like(x) for x in xs]
    say("q3 batch apply", bt.config)
    bt.apply(xs, ys)
    i = 0
    for p, wl, op in zip(probs, wls, ops):
        for r in range(3):
            y = host(ys[i])
            yref = op.matvec(wl.vectors[r])
            say("q3 mesh", wl.mesh.ncells[0], "rhs", r, f"err {rel(y, yref):.2e} max {rel_max(y, yref):.2e}")
            assert rel(y, yref) < 1e-12 and rel_max(y, yref) < 1e-12
            assert rel(y, host(p.apply(xs[i]))) < 1e-13
            i += 1
    first = [y.clone() for y in ys]
    for _ in range(2):
        bt.apply(xs, ys)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(first, ys))


def test_batch_q3_cg_fp64_matches_oracle():
    """Lockstep FP64 PCG of Q3 systems (three meshes, two right-hand sides
    each: the manufactured sine load of the mesh's sphere and the phi-free sine
    load): each reaches the oracle's direct solution with its true residual
    (oracle CSR) below rtol, in the oracle PCG's iteration count +-2."""
    wls = W.batch_meshes(sizes=(4, 6, 5), nrhs=2, k=3)
    probs, systems = [], []
    for wl in wls:
        m = wl.mesh
        p = vpp.Problem.from_mesh(m)
        p.set_phi(dev(wl.phi))
        probs.append(p)
        op = oracle.Operator(m, phi=wl.phi)
        for b in (oracle.manufactured_sine_rhs(m, wl.extra["radius"], m.eps), oracle.sine_load(m)):
            systems.append((op, b))
    bt = vpp.Batch(probs, [2] * len(probs))
    bs = [dev(b) for _, b in systems]
    xs = [torch.zeros_like(b) for b in bs]
    say("q3 batch cg", bt.config)
    infos = bt.cg_solve(bs, xs, rtol=1e-10, check_every=4)
    for i, ((op, b), inf) in enumerate(zip(systems, infos)):
        x = host(xs[i])
        pref = spla.spsolve(op.to_scipy().tocsc(), b)
        res = np.linalg.norm(b - op.matvec(x)) / np.linalg.norm(b)
        _, oinf = op.pcg(b, rtol=1e-10)
        say("q3 system", i, inf["iterations"], "oracle", oinf["iterations"], f"res {res:.2e}")
        assert inf["status"] == 0
        assert res < 1e-10 * 1.01
        assert rel(x, pref) < 1e-8
        assert abs(inf["iterations"] - oinf["iterations"]) <= 2


def test_batch_rejects_degree_four():
    wl = W.batch_meshes(sizes=(3,), nrhs=1, k=4)[0]
    p = vpp.Problem.from_mesh(wl.mesh)
    p.set_phi(dev(wl.phi))
    with pytest.raises(vpp.VppError) as e:
        vpp.Batch([p], [1])
    assert "degrees 2 and 3" in str(e.value)


@pytest.mark.parametrize("k", [2, 3])
def test_batch_with_mass_shift_equals_single(k):
    """A batch of two meshes, one with the mass shift mu M (set before the batch
    is created) and one without: every output equals the single-problem apply
    of its problem (which the oracle pins with and without the shift), and the
    lockstep PCG of the shifted systems reaches the single solve's iterate."""
    wls = W.batch_meshes(sizes=(5, 7), nrhs=2, k=k)
    probs = []
    for i, wl in enumerate(wls):
        p = vpp.Problem.from_mesh(wl.mesh)
        p.set_phi(dev(wl.phi))
        if i == 0:
            p.set_mass(0.75)
        probs.append(p)
    bt = vpp.Batch(probs, [2, 2])
    xs = [dev(wl.vectors[r]) for wl in wls for r in range(2)]
    ys = [torch.empty_like(x) for x in xs]
    say("mass batch", k, bt.config)
    bt.apply(xs, ys)
    for i, p in enumerate(q for q in probs for _ in range(2)):
        assert rel(host(ys[i]), host(p.apply(xs[i]))) < 1e-13
    bs = [p.apply(x) for p, x in zip((q for q in probs for _ in range(2)), xs)]
    sol = [torch.zeros_like(b) for b in bs]
    infos = bt.cg_solve(bs, sol, rtol=1e-10)
    for i, (p, inf) in enumerate(zip((q for q in probs for _ in range(2)), infos)):
        x1, inf1 = p.cg_solve(bs[i], rtol=1e-10)
        assert inf["status"] == 0 and abs(inf["iterations"] - inf1["iterations"]) <= 1
        assert rel(host(sol[i]), host(x1)) < 1e-8


@pytest.mark.timeout(600)
def test_q3_batch_bench_workload_against_oracle():
    """The Q3 batch that bench.py times (8 meshes of 8..32 cells per side, 4
    seeded right-hand sides each, one persistent batched apply in the tuned
    configuration): every output against the oracle at 1e-12 relative - all
    rows on the meshes up to 12^3 (CSR), 1500 seeded rows plus every 997th row
    on the larger ones (row by row)."""
    wls = W.batch_meshes(sizes=(8, 10, 12, 14, 16, 20, 24, 32), nrhs=4, k=3)
    probs, xs = [], []
    for wl in wls:
        p = vpp.Problem.from_mesh(wl.mesh)
        p.set_phi(dev(wl.phi))
        probs.append(p)
        xs += [dev(v) for v in wl.vectors]
    ys = [torch.empty_like(x) for x in xs]
    bt = vpp.Batch(probs, [4] * len(probs))
    say("q3 bench batch apply", bt.config)
    bt.apply(xs, ys)
    torch.cuda.synchronize()
    rng = np.random.default_rng(78)
    i = 0
    for wl in wls:
        m = wl.mesh
        full = m.ncells[0] <= 12
        op = oracle.Operator(m, phi=wl.phi) if full else None
        rows = None if full else np.unique(np.concatenate([rng.choice(m.ndofs, 1500, replace=False),
                                                            np.arange(0, m.ndofs, 997)]))
        for r in range(4):
            y, x = host(ys[i]), wl.vectors[r]
            if full:
                yref = op.matvec(x)
                err, errm = rel(y, yref), rel_max(y, yref)
            else:
                yr = oracle.apply_rows(m, wl.phi, x, rows)
                err, errm = rel(y[rows], yr), rel_max(y[rows], yr)
            say("q3 bench mesh", m.ncells[0], "rhs", r, f"err {err:.2e} max {errm:.2e}")
            assert err < 1e-12 and errm < 1e-12
            i += 1
