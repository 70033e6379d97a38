"""Host-side checks of the C ABI: the shared library loads and exports every
function that include/dbs.h declares (no GPU work is started)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2003_08374_amd", "libdbs.so")


def declared_functions():
    src = open(os.path.join(ROOT, "include", "dbs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dbs_[a-z_]+)\s*\(", src)))


def test_header_declares_the_step_interface():
    names = declared_functions()
    for n in ("dbs_create", "dbs_set_static", "dbs_set_state", "dbs_step", "dbs_get_state",
              "dbs_destroy", "dbs_debug_pressure_solve"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdbs.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdbs.so not built")
def test_binding_lists_match_header():
    from paper_2003_08374_amd import dbs
    assert sorted(dbs.EXPORTS) == declared_functions()


def test_product_package_does_not_reach_the_oracle():
    pkg = os.path.join(ROOT, "paper_2003_08374_amd")
    for dp, _, fs in os.walk(pkg):
        for f in fs:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dp, f)).read()
                assert "dbs_oracle" not in txt and "import oracle" not in txt, f


def test_batch_rejects_mixed_physics_before_touching_the_device():
    """A batch shares one set of physics and controls: a sample that differs
    is refused by the binding (no device call is made for it)."""
    from paper_2003_08374_amd import dbs, workloads as W
    a = W.droplet(shape=(8, 8, 1), radius_cells=3)
    b = a.replace(sigma=0.03)
    with pytest.raises(ValueError):
        dbs.BatchSolver([a, b])
