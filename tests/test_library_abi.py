"""The C-ABI library loads (no GPU needed), exports every function that
include/re.h declares, and rejects invalid arguments before touching the
device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(re_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def R():
    from paper_0812_1633_amd import re as R
    if not os.path.exists(R.LIB_PATH):
        from paper_0812_1633_amd import build
        build.build()
    R.lib()
    return R


def test_exports_every_declared_symbol(R):
    names = declared_functions()
    assert "re_create" in names and "re_step" in names and len(names) >= 15
    lib = ctypes.CDLL(R.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("kw,msg", [
    (dict(N=[256, 1], T=[0.7, 0.8]), "N_atoms"),
    (dict(N=[256, 256], T=[0.8, 0.7]), "ascending"),
    (dict(N=[256, 256], T=[0.0, 0.7]), "T_ladder"),
    (dict(N=[100], T=[1.0]), "L/2"),
    (dict(N=[256], T=[1.0], dt=0.0), "dt"),
    (dict(N=[256], T=[1.0], Nx=0), "N_x"),
    (dict(N=[256], T=[1.0], rho=-1.0), "rho"),
    (dict(N=[6_000_000], T=[1.0]), "2^32 bytes"),
])
def test_invalid_arguments(R, kw, msg):
    args = dict(rho=0.8442, rc=2.5, skin=0.3, dt=0.005, Nx=10)
    args.update(kw)
    with pytest.raises(R.ReError) as e:
        R.Engine(args["N"], args["T"], args["rho"], args["rc"], args["skin"], args["dt"], args["Nx"], 1)
    assert e.value.code == R.RE_EINVAL
    assert msg in str(e.value)


def test_invalid_options(R):
    for kw in (dict(threads_per_atom=3), dict(block_size=100), dict(threads_per_atom_per_replica=[6])):
        with pytest.raises(R.ReError) as e:
            R.Engine([256], [1.0], 0.8442, 2.5, 0.3, 0.005, 10, 1, **kw)
        assert e.value.code == R.RE_EINVAL
    with pytest.raises(R.ReError) as e:
        R.Engine([256], [1.0], 0.8442, 2.5, 0.3, 0.005, 10, 1, form="plain", exchange="async")
    assert e.value.code == R.RE_EINVAL
