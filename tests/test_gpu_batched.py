"""Batched multi-cell path: several cells of different grid sizes in one
call, eagerly and through a replayed HIP graph; the autotuner."""
import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
from paper_1801_09263_amd import lace  # noqa: E402
from paper_1801_09263_amd.batch import MultiCell  # noqa: E402
from paper_1801_09263_amd.session import CellSession  # noqa: E402

pytestmark = pytest.mark.gpu

FP64, FP32 = lace.LACE_FP64, lace.LACE_FP32


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def make_cells():
    out = []
    for (L, n, ecut, n_orb, seed) in ((9.0, 16, 6.0, 5, 1), (10.0, 24, 15.0, 8, 2),
                                      (12.0, 48, 20.0, 12, 3)):
        m = synth.miller_sphere(L, ecut)
        c = synth.random_orbitals(m, L, n_orb, synth.rng_for(80, seed))
        out.append((dict(L=L, n=n, miller=m, s_thr=0.0), c))
    L, n, ecut = 16.0, 32, 15.0
    m = synth.miller_sphere(L, ecut)
    c = synth.gaussian_orbitals(m, L, 16, 8, synth.rng_for(90))
    out.append((dict(L=L, n=n, miller=m, s_thr=2e-3), c))
    return out


def single_results(cells, prec):
    res = []
    for cell, coeffs in cells:
        s = CellSession(cell, coeffs.shape[0], prec)
        s.set_orbitals(coeffs)
        s.apply_exchange(cell["s_thr"])
        s.build_ace("avg")
        torch.cuda.synchronize()
        res.append(dict(w=s.w.clone(), e_x=s.e_x.clone(), xi=s.xi.clone(),
                        m=s.m.clone(), kept=s.n_kept))
        s.close()
    return res


def check_same(mc, ref):
    for k, r in enumerate(ref):
        j = mc.jobs[k]
        assert mc.n_kept[k] == r["kept"]
        assert torch.equal(j["w_g"], r["w"]), f"W of job {k}"
        assert torch.equal(j["e_x"], r["e_x"]), f"E_x of job {k}"
        assert torch.equal(j["m_out"], r["m"]), f"M of job {k}"
        assert torch.equal(j["xi_g"], r["xi"]), f"xi of job {k}"


@pytest.mark.parametrize("prec", [FP32, FP64], ids=["fp32", "fp64"])
def test_batched_equals_alone(prec):
    say(f"batched vs alone prec={prec}")
    cells = make_cells()
    ref = single_results(cells, prec)
    mc = MultiCell([c for c, _ in cells], [x.shape[0] for _, x in cells], prec)
    for k, (_, coeffs) in enumerate(cells):
        mc.set_orbitals(k, coeffs)
    mc.run(graph=False)
    torch.cuda.synchronize()
    check_same(mc, ref)
    # and the screened cell against the oracle
    cell, coeffs = cells[3]
    pairs = O.kept_pairs(O.overlap_of_moduli(
        O.orbitals_on_grid(coeffs, cell["miller"], cell["L"], cell["n"]),
        cell["L"]), cell["s_thr"])
    res = O.run_path(coeffs, cell["miller"], cell["L"], cell["n"], pairs=pairs)
    tol = 1e-5 if prec == FP32 else 1e-11
    assert rel(mc.jobs[3]["w_g"].cpu().numpy(), res["W_pw"]) <= tol
    mc.close()


def test_graph_replays_match_eager():
    """The captured graph, replayed three times with eager work and
    synchronizations in between, reproduces the eager results bitwise; a
    change of orbitals (same pair lists) is picked up by the replay."""
    say("graph replays")
    cells = make_cells()
    ref = single_results(cells, FP32)
    mc = MultiCell([c for c, _ in cells], [x.shape[0] for _, x in cells], FP32)
    for k, (_, coeffs) in enumerate(cells):
        mc.set_orbitals(k, coeffs)
    stream = torch.cuda.Stream()
    for rep in range(3):
        for j in mc.jobs:
            j["w_g"].zero_()
            j["xi_g"].zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            mc.run(graph=True, stream=stream)
        stream.synchronize()
        check_same(mc, ref)
        # eager work between replays
        junk = torch.randn(1 << 20, device="cuda")
        (junk * 2).sum().item()
        single_results(cells[:1], FP32)
        torch.cuda.synchronize()
    # new orbitals in an unscreened job: same schedule, graph replayed
    cells2 = list(cells)
    m = cells[1][0]["miller"]
    c_new = synth.random_orbitals(m, 10.0, 8, synth.rng_for(81))
    cells2[1] = (cells[1][0], c_new)
    mc.set_orbitals(1, c_new)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        mc.run(graph=True, stream=stream)
    stream.synchronize()
    ref2 = single_results(cells2[1:2], FP32)[0]
    assert torch.equal(mc.jobs[1]["w_g"], ref2["w"])
    # new orbitals in the screened job: the replay screens them on the
    # device (new pair list, new schedule) and matches the eager call
    cell3 = cells[3][0]
    c3 = synth.gaussian_orbitals(cell3["miller"], cell3["L"],
                                 cells[3][1].shape[0],
                                 cells[3][1].shape[0] // 2, synth.rng_for(82))
    cells2[3] = (cell3, c3)
    mc.set_orbitals(3, c3)
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        mc.run(graph=True, stream=stream)
    stream.synchronize()
    ref3 = single_results(cells2[3:4], FP32)[0]
    say(f"  screened job: kept {mc.n_kept[3]} (was {ref[3]['kept']}), "
        f"eager {ref3['kept']}")
    assert mc.n_kept[3] == ref3["kept"]
    assert torch.equal(mc.jobs[3]["w_g"], ref3["w"])
    assert torch.equal(mc.jobs[3]["xi_g"], ref3["xi"])
    mc.close()


def test_autotune_picks_a_candidate_and_stays_correct():
    say("autotune")
    L, n, ecut, n_orb = 12.0, 48, 20.0, 24
    m = synth.miller_sphere(L, ecut)
    coeffs = synth.random_orbitals(m, L, n_orb, synth.rng_for(82))
    cell = dict(L=L, n=n, miller=m, s_thr=0.0)
    mc = MultiCell([cell], [n_orb], FP32)
    mc.set_orbitals(0, coeffs)
    cands = mc.autotune(0)
    say("  candidates", cands)
    stage1 = [c for c in cands if c[2] == 0 and c[3] == 0]
    stage2 = cands[len(stage1):]
    assert cands[:len(stage1)] == stage1
    assert len(stage1) == 12     # 4 batch sizes x 3 xy schedules
    assert all(c[4] > 0 for c in cands)
    # stage 2 varies the z tile and the radix order of one stage-1
    # candidate (the fastest over its whole schedule; the other stage-1
    # times may cover only their first batches, so they are not compared)
    bases = {(c[0], c[1]) for c in stage2}
    assert stage2 and len(bases) == 1
    assert any((c[0], c[1]) in bases for c in stage1)
    assert {(c[2], c[3]) for c in stage2} <= {(1, 0), (2, 0), (0, 1)}
    chosen = lace.lace_get_tuning(mc.plan, 0)
    assert chosen in [tuple(c[:4]) for c in cands]
    t_chosen = min(c[4] for c in cands if tuple(c[:4]) == chosen)
    assert all(t_chosen <= c[4] for c in stage2)
    mc.run()
    torch.cuda.synchronize()
    res = O.run_path(coeffs, m, L, n)
    assert rel(mc.jobs[0]["w_g"].cpu().numpy(), res["W_pw"]) <= 1e-5
    # every candidate schedule gives the same W to FP32 rounding
    w0 = mc.jobs[0]["w_g"].clone()
    for ppb_c, plane_c, z_c, r_c, _ in cands:
        lace.lace_set_tuning(mc.plan, 0, ppb_c, plane_c, z_c, r_c)
        mc.run()
        torch.cuda.synchronize()
        assert rel(mc.jobs[0]["w_g"].cpu().numpy(), w0.cpu().numpy()) <= 2e-6
    mc.close()


def test_tuning_rejects_bad_values():
    cell = dict(L=10.0, n=24, miller=synth.miller_sphere(10.0, 15.0))
    plan = lace.lace_plan_create([cell], FP32)
    for ppb, pl, zt, ro in ((0, 1, 0, 0), (65, 1, 0, 0), (8, 3, 0, 0),
                            (8, -1, 0, 0), (8, 2, 3, 0), (8, 2, -1, 0),
                            (8, 2, 0, 2)):
        with pytest.raises(lace.LaceError):
            lace.lace_set_tuning(plan, 0, ppb, pl, zt, ro)
    plan.close()


def test_batched_gamma_equals_alone():
    """Real-orbital packing through the batched path: three localized cells
    of different sizes, bitwise equal to running each alone."""
    say("batched gamma vs alone")
    cells = []
    for (L, n, ecut, n_orb, seed) in ((12.0, 48, 20.0, 14, 1),
                                      (16.0, 32, 15.0, 16, 2),
                                      (9.0, 24, 12.0, 9, 3)):
        m = synth.miller_sphere(L, ecut)
        c = synth.gaussian_orbitals(m, L, n_orb, (n_orb + 1) // 2,
                                    synth.rng_for(85, seed))
        cells.append((dict(L=L, n=n, miller=m, s_thr=1e-3), c))
    prec = lace.LACE_FP32_GAMMA
    ref = single_results(cells, prec)
    mc = MultiCell([c for c, _ in cells], [x.shape[0] for _, x in cells], prec)
    for k, (_, coeffs) in enumerate(cells):
        mc.set_orbitals(k, coeffs)
    mc.run(graph=False)
    torch.cuda.synchronize()
    check_same(mc, ref)
    mc.close()
