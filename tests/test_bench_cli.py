"""CPU checks of the benchmark's contract: it measures one GPU and says so for
any other count, and the committed HBM-traffic summary it reads is well formed
(the value is used only while its recorded source digest matches the sort's
sources; otherwise the benchmark reports the traffic as null)."""
import importlib.util
import json
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_traffic_summary_is_well_formed():
    bench = _bench()
    with open(os.path.join(ROOT, bench.TRAFFIC_FILE) if not os.path.isabs(bench.TRAFFIC_FILE)
              else bench.TRAFFIC_FILE) as f:
        text = f.read()
    m = re.search(r"^traffic_json: (\{.*\})$", text, re.M)
    assert m, "no traffic_json line"
    t = json.loads(m.group(1))
    for k in ("kernel", "n_log2", "hbm_bytes_per_launch", "algorithmic_bytes_per_launch", "fetch_scale",
              "write_scale", "sources_sha256"):
        assert k in t, k
    assert t["kernel"] == "k_radix_scatter" and t["n_log2"] == 26
    # The method's pair passes move 4-byte keys; the sort behind the benchmark
    # stores 16-bit keys between passes, so its launches move 10n and 12n
    # bytes against 12n and 16n algorithmic (0.79), plus any waste.
    assert 0.7 < t["hbm_bytes_per_launch"] / t["algorithmic_bytes_per_launch"] < 1.5
    assert re.fullmatch(r"[0-9a-f]{64}", t["sources_sha256"])
    # the digest function reads the sources the summary was taken from
    assert re.fullmatch(r"[0-9a-f]{64}", bench.sources_digest(bench.SCATTER_SOURCES))
