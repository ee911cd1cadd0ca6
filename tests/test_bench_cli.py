"""bench.py's command line on the host (no GPU): more than one GPU is refused
with a message, and the traffic table belongs to the kernel sources it names."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and "--gpus 2" in p.stderr
    assert p.stdout.strip() == ""


def test_traffic_table_names_kernel_sources():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    h = b.kernel_source_hash()
    assert len(h) == 16 and all(c in "0123456789abcdef" for c in h)
    for key, t in b.TRAFFIC.items():
        assert t["fetch"] > 0 and t["write"] > 0 and len(t["src"]) == 16, key
