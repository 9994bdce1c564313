"""The benchmark's command-line contract and the consistency of the committed
measurement files with the current sources (CPU only).

- `bench.py --gpus N` with N > 1 exits with status 2 and says why, before it
  touches a GPU.
- The rocprofv3 summaries the bench line quotes (kernel trace, HBM traffic)
  were taken on the current kernel sources, and the committed tuning cache
  holds entries for the current library sources, so the bench line reports
  counter traffic and runs the tuned launch shapes.
"""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1801_03863_amd import build  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_profiles_match_the_kernel_sources():
    digest = bench.kernel_source_digest()
    assert re.fullmatch(r"[0-9a-f]{16}", digest)
    assert bench.read_traffic(digest) is not None, "traffic summary taken on other kernel sources"
    assert bench.read_valu(digest) is not None, "VALU summary taken on other kernel sources"
    # every committed summary was taken on the current kernel sources
    names = sorted(os.listdir(os.path.join(ROOT, "profiles")))
    assert names
    for name in names:
        txt = open(os.path.join(ROOT, "profiles", name)).read()
        assert "kernel_source_sha256_16: %s" % digest in txt, name


def test_tuning_cache_matches_the_library_sources():
    sid = build.source_id()
    path = os.path.join(ROOT, "paper_1801_03863_amd", "tune_cache_gfx950.txt")
    keys = [line.split()[0] for line in open(path) if line.strip()]
    assert keys and all(k.startswith(sid + "|") for k in keys)
    # the benchmark's headline workload is among them
    assert any("|prec1|coll0|bc2|n1|4096x4096|" in k for k in keys)
