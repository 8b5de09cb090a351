"""bench.py on the host: the one-GPU guard and the recorded HBM traffic figures
(no GPU needed)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_traffic_records_are_complete():
    path = os.path.join(ROOT, "profiles", "traffic.json")
    recs = json.load(open(path))
    assert recs
    for key, ent in recs.items():
        workload, _, prec = key.partition("|")
        assert ent["precision"] == prec and prec in ("p64", "p32", "pb3", "pb6")
        assert len(ent["source_hash"]) == 16
        # copy calibration: FETCH_SIZE counts half the bytes read, WRITE_SIZE all written
        assert 1.9 < ent["fetch_factor"] < 2.1 and 0.95 < ent["write_factor"] < 1.05
        assert os.path.exists(os.path.join(ROOT, ent["summary"])), ent["summary"]
        for k in ("blocks", "contract"):
            e = ent[k]
            assert e["bytes_per_launch"] > 0
            assert abs(e["fetch_bytes"] + e["write_bytes"] - e["bytes_per_launch"]) <= 1e-6 * e["bytes_per_launch"]
        # the block kernel reads both propagators at least once (4608 bytes per
        # site and time slice of complex128, 2304 of complex64)
        sites, esz = {"3He-16^3x32": (16 ** 3 * 32, 4608), "4He-24^3x48": (24 ** 3 * 48, 4608),
                      "batch64-16^3x32": (64 * 16 ** 3 * 32, 2304)}[workload]
        assert ent["blocks"]["fetch_bytes"] >= 0.99 * esz * sites
