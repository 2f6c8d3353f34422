"""Serving loop: each job's results are the same alone and in the mix of
concurrently running jobs, and admission respects the memory budget."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
from paper_1801_09263_amd import lace  # noqa: E402
from paper_1801_09263_amd.serving import Job, JobClass, Server, summarize  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def classes():
    specs = [(12.0, 48, 32), (16.0, 64, 64)]
    raw = synth.serving_classes(seed=3, n_variants=3, specs=specs)
    out = []
    for c in raw:
        pool = [torch.tensor(v, device="cuda") for v in c["variants"]]
        cell = {k: c[k] for k in ("L", "n", "miller", "s_thr", "rc")}
        out.append(JobClass(c["name"], cell, c["n_orb"], pool))
    return out


def make_jobs(n_jobs, rate, seed=5):
    spec = synth.serving_stream(n_jobs, 2, [3, 3], rate=rate, n_steps=2,
                                large_fraction=0.0, seed=seed)
    return [Job(jid, t, cls, var) for jid, t, cls, var in spec]


@pytest.mark.parametrize("inner,align", [(1, False), (3, True)],
                         ids=["plain", "aligned"])
def test_results_same_alone_and_in_the_mix(classes, inner, align):
    say(f"serving: mix of 8 jobs on 3 slots vs each alone (inner {inner}, "
        f"align {align})")
    mix = Server(classes, lace.LACE_FP32, n_slots=3, keep_xi=True,
                 inner=inner, align=align)
    jobs = mix.run(make_jobs(8, rate=400.0))
    mix.close()
    assert all(j.done > j.admit >= j.arrival for j in jobs)
    # jobs really overlapped on the device
    overl = sum(1 for a in jobs for b in jobs
                if a.jid < b.jid and a.admit < b.done and b.admit < a.done)
    say(f"  overlapping job pairs: {overl}")
    assert overl > 0
    alone = Server(classes, lace.LACE_FP32, n_slots=1, keep_xi=True,
                   inner=inner, align=align)
    for j in jobs:
        solo = Job(j.jid, 0.0, j.cls, j.variants)
        alone.run([solo])
        assert solo.kept == j.kept
        assert solo.e_x == j.e_x, f"E_x of job {j.jid}"
        assert np.array_equal(solo.xi_host, j.xi_host), f"xi of job {j.jid}"
    alone.close()
    s = summarize(jobs, 400.0)
    say("  ", s)
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_admission_respects_memory_budget(classes):
    say("serving: memory-limited admission")
    big = max(c.footprint for c in classes) if classes[0].footprint else None
    probe = Server(classes, lace.LACE_FP32, n_slots=1)
    fps = [c.footprint for c in probe.classes]
    probe.close()
    budget = int(1.5 * max(fps))
    srv = Server(classes, lace.LACE_FP32, n_slots=4, hbm_budget=budget)
    jobs = srv.run(make_jobs(10, rate=400.0, seed=6))
    srv.close()
    del big
    events = sorted([(j.admit, +fps[j.cls]) for j in jobs]
                    + [(j.done, -fps[j.cls]) for j in jobs],
                    key=lambda e: (e[0], e[1]))
    used = 0
    for _, d in events:
        used += d
        assert used <= budget
