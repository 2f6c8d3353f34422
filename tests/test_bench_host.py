"""Host-side parts of bench.py: the per-pair byte model, the counter
summary that writes the traffic figures, and the one-GPU guard."""
import json
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_pair_byte_model():
    # off-diagonal pair: 3, 2, 7 orbital grids; diagonal 2, 2, 4
    assert bench.pass_alg_bytes(0, 1, 0, 4, 10) == 3 * 4 * 10
    assert bench.pass_alg_bytes(1, 1, 0, 4, 10) == 2 * 4 * 10
    assert bench.pass_alg_bytes(2, 1, 0, 4, 10) == 7 * 4 * 10
    assert bench.pass_alg_bytes(0, 0, 1, 4, 10) == 2 * 4 * 10
    assert bench.pass_alg_bytes(2, 0, 1, 8, 10) == 4 * 8 * 10
    assert bench.pass_alg_bytes(2, 5, 3, 4, 7) == (7 * 5 + 4 * 3) * 4 * 7


def _counter_db(path, rows):
    db = sqlite3.connect(path)
    db.execute("create table counters_collection (kernel_name text, "
               "dispatch_id integer, value real)")
    db.executemany("insert into counters_collection values (?, ?, ?)", rows)
    db.commit()
    db.close()


def test_write_traffic_scaling(tmp_path):
    kib = 1 << 20   # the 1 GiB copy in KiB
    names = ["void lace::k_half<float, 8, ProQuadD<float>>(args)",
             "void lace::k_zconv<float, 8>(args)",
             "void lace::k_half<float, 8, EpiAccQuadD<float>>(args)"]
    fetch, write = [("__amd_rocclr_copyBuffer", 1, kib / 2),
                    ("__amd_rocclr_copyBuffer", 2, 3.0)], \
                   [("__amd_rocclr_copyBuffer", 1, kib),
                    ("__amd_rocclr_copyBuffer", 2, 1.0)]
    d = 10
    for k, n in enumerate(names):
        for b in range(2):   # two launches per pass, split over two rows
            fetch += [(n, d, 100.0 * (k + 1)), (n, d, 100.0 * (k + 1))]
            write += [(n, d, 50.0 * (k + 1))]
            d += 1
    _counter_db(tmp_path / "f.db", fetch)
    _counter_db(tmp_path / "w.db", write)
    sample = {"pmc_sample": "ok", "n_kept": 10, "n_orb": 4, "n": 2,
              "launches": [2, 2, 2], "alg_bytes": [1e6, 2e6, 3e6]}
    (tmp_path / "s.log").write_text("noise\n" + json.dumps(sample) + "\n")
    out = tmp_path / "traffic.json"
    res = bench.write_traffic(str(tmp_path / "f.db"), str(tmp_path / "w.db"),
                              str(tmp_path / "s.log"), str(out))
    assert json.loads(out.read_text()) == json.loads(json.dumps(res))
    assert res["fetch_scale"] == pytest.approx(2.0)
    assert res["write_scale"] == pytest.approx(1.0)
    assert res["kernel_source_hash"] == bench.kernel_source_hash()
    for k in range(3):
        p = res["passes"][str(k)]
        assert p["launches"] == 2
        # per dispatch: fetch 2 x 100 (k+1) KiB scaled by 2, write 50 (k+1)
        assert p["fetch_bytes"] == pytest.approx(400.0 * (k + 1) * 1024)
        assert p["write_bytes"] == pytest.approx(50.0 * (k + 1) * 1024)
        assert p["moved_bytes_per_launch"] == pytest.approx(sample["alg_bytes"][k] / 2)
        alg = bench.pass_alg_bytes(k, 6, 4, 4, 8) / 2
        assert p["alg_bytes_per_launch"] == pytest.approx(alg)
        assert p["ratio"] == pytest.approx(p["bytes_per_launch"] / p["moved_bytes_per_launch"])


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
