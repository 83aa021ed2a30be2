"""The C-ABI library loads, exports every entry point include/pmp.h declares,
and rejects bad arguments on the host before touching a device.  Runs without
a GPU (no compute calls)."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"PMP_API\s+[\w\s\*]+?\b(pmp_\w+)\s*\(", text)
    return names


def test_header_declares_the_four_named_entry_points():
    names = _declared()
    for n in ("pmp_preprocess", "pmp_eval_population", "pmp_ga_step", "pmp_solve"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1610_10061_amd as pm
    L = pm.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(_declared()) == set(pm.EXPORTS)


def test_status_strings():
    import paper_1610_10061_amd as pm
    L = pm.lib()
    assert L.pmp_status_str(0) == b"ok"
    assert L.pmp_status_str(4) == b"infeasible chromosome"


@pytest.mark.parametrize("shape,p", [((3, 1), 1), ((4, 5), 0), ((4, 5), 5), ((0, 5), 2),
                                     ((2, 65536), 3)])
def test_preprocess_rejects_bad_sizes(shape, p):
    """Sizes rejected before any device call (m above 65535 included: the
    facility indices of Pi' are 16-bit)."""
    import paper_1610_10061_amd as pm
    d = np.zeros(shape, np.int32)
    with pytest.raises(pm.PmpError) as e:
        pm.pmp_preprocess(d, p)
    assert e.value.status == pm.PMP_EINVAL


def test_preprocess_async_needs_device_input():
    """PMP_ASYNC leaves the work on a stream after the call returns, so a
    host matrix (copied by the call) is refused before any device work."""
    import ctypes as C
    import paper_1610_10061_amd as pm
    d = np.arange(12, dtype=np.int32).reshape(3, 4)
    out = C.c_void_p()
    st = pm.lib().pmp_preprocess(d.ctypes.data_as(C.c_void_p), 4, 3, 4, 2, pm.PMP_ASYNC, None,
                                 C.byref(out))
    assert st == pm.PMP_EINVAL and not out.value


def test_preprocess_rejects_negative_distance_on_host():
    import paper_1610_10061_amd as pm
    d = np.ones((4, 6), np.int32)
    d[2, 3] = -1
    with pytest.raises(pm.PmpError) as e:
        pm.pmp_preprocess(d, 2)
    assert e.value.status == pm.PMP_EINVAL
    assert "d[2][3]" in str(e.value)


def test_null_handles_rejected():
    import paper_1610_10061_amd as pm
    L = pm.lib()
    assert L.pmp_eval_population(None, None, 1, None, None, 0, None) == pm.PMP_EINVAL
    assert L.pmp_ga_step(None, 1, None) == pm.PMP_EINVAL
    assert L.pmp_instance_info(None, None, None, None, None, None) == pm.PMP_EINVAL
    assert L.pmp_batch_step(None, 1, None) == pm.PMP_EINVAL
    assert L.pmp_batch_autotune(None, None, None) == pm.PMP_EINVAL
    assert L.pmp_batch_profile(None, 1) == pm.PMP_EINVAL
    L.pmp_instance_destroy(None)
    L.pmp_ga_destroy(None)
    L.pmp_batch_destroy(None)


def test_ga_params_rejected_before_allocation():
    import ctypes as C
    import paper_1610_10061_amd as pm
    L = pm.lib()
    out = C.c_void_p()
    fake = C.c_void_p(1)  # never dereferenced: validation fails first
    for P, NT, G in ((0, 1, 1), (96, 48, 1), (64, 128, 1), (64, 64, 0), (2048, 2048, 1)):
        prm = pm.GaParams(1, P, NT, G, 0, 0, 0)
        assert L.pmp_ga_create(fake, C.byref(prm), C.byref(out)) == pm.PMP_EINVAL


def test_oracle_and_product_share_nothing():
    """The oracle and the GPU path import nothing from each other."""
    import ast
    for pkg, other in (("oracle", "paper_1610_10061_amd"), ("paper_1610_10061_amd", "oracle")):
        for dp, _, fs in os.walk(os.path.join(ROOT, pkg)):
            for f in fs:
                path = os.path.join(dp, f)
                if f.endswith(".py"):
                    for node in ast.walk(ast.parse(open(path).read())):
                        if isinstance(node, ast.Import):
                            assert all(not a.name.startswith(other) for a in node.names), path
                        if isinstance(node, ast.ImportFrom) and node.module:
                            assert not node.module.startswith(other), path
                elif f.endswith((".c", ".h", ".hip", ".hpp", ".cpp")):
                    incs = [ln for ln in open(path) if ln.lstrip().startswith("#include")]
                    banned = ("oracle",) if pkg != "oracle" else ("pmp.h", "common.hpp", "philox.hpp")
                    assert not [ln for ln in incs if any(b in ln for b in banned)], path


def test_apsp_rejects_bad_arguments_before_any_device_work():
    import ctypes as C
    import paper_1610_10061_amd as pm
    w = np.zeros((4, 4), np.int32)
    d = np.zeros((4, 4), np.int32)
    L = pm.lib()
    vp = pm._vp
    assert L.pmp_apsp(None, 4, 4, d.ctypes.data_as(vp), 4, 0, None) == pm.PMP_EINVAL
    assert L.pmp_apsp(w.ctypes.data_as(vp), 4, 0, d.ctypes.data_as(vp), 4, 0, None) == pm.PMP_EINVAL
    assert L.pmp_apsp(w.ctypes.data_as(vp), 3, 4, d.ctypes.data_as(vp), 4, 0, None) == pm.PMP_EINVAL
    assert L.pmp_apsp(w.ctypes.data_as(vp), 4, 40000, d.ctypes.data_as(vp), 40000, 0,
                      None) == pm.PMP_EINVAL
