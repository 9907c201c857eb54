"""Host-side checks of the C ABI that need no GPU: the library builds, loads,
and exports every entry point that include/sscs.h declares; the binding's
struct layouts match the header's field lists."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sscs.h")


def _declared():
    txt = open(HEADER).read() + open(os.path.join(ROOT, "include", "sscs_mlp.h")).read()
    return sorted(set(re.findall(r"\b(sscs_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["sscs_create", "sscs_solve", "sscs_destroy", "sscs_linear_step", "sscs_project_dual_cone",
                 "sscs_residual", "sscs_batch_create", "sscs_batch_solve", "sscs_batch_destroy"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1903_06477_amd import sscs
    if not os.path.exists(sscs.LIB_PATH):
        from paper_1903_06477_amd import build
        build.build()
    L = ctypes.CDLL(sscs.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name
    assert sorted(sscs.EXPORTS) == _declared()


def test_struct_fields_match_header():
    from paper_1903_06477_amd import sscs
    txt = open(HEADER).read()

    def fields(struct_name):
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + struct_name + ";", txt).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        names = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            for part in decl.split(","):
                tok = re.findall(r"[A-Za-z_][A-Za-z_0-9]*", part)
                names.append(tok[-1])
        return names

    assert [f for f, _ in sscs._Data._fields_] == fields("sscs_data")
    assert [f for f, _ in sscs._Cone._fields_] == fields("sscs_cone")
    assert [f.rstrip("_") for f, _ in sscs._Settings._fields_] == fields("sscs_settings")
    assert [f for f, _ in sscs._Info._fields_] == fields("sscs_info")


def test_default_settings_and_error_strings():
    from paper_1903_06477_amd import sscs
    L = sscs.lib()
    st = sscs._Settings()
    assert L.sscs_default_settings(ctypes.byref(st)) == 0
    assert st.eps == 1e-6 and st.mem == 5 and st.direction == 1
    # converging defaults of the Algorithm 1 inputs the paper leaves open; the
    # binding's defaults are the library's
    assert (st.c1, st.q, st.lambda_, st.check_every, st.workgroups) == (0.9999, 0.999, 1.5, 1, 0)
    py = sscs.Settings().to_c()
    for f, _ in sscs._Settings._fields_:
        if f != "c0":
            assert getattr(py, f) == getattr(st, f), f
    assert L.sscs_error_string(-1) == b"invalid argument"
    assert L.sscs_default_settings(None) == -1


def test_create_rejects_bad_input_before_touching_the_device():
    # validation happens on the host, before any HIP call
    import numpy as np
    import scipy.sparse as sp
    from paper_1903_06477_amd import sscs
    from paper_1903_06477_amd.generators import Cone, Problem
    A = sp.csr_matrix(np.ones((3, 2)))
    bad = Problem(A=A, b=np.ones(3), c=np.ones(2), cone=Cone(l=2))        # cone rows 2 != m 3
    with pytest.raises(sscs.SSCSError, match="invalid"):
        sscs.Solver(bad)
    bad2 = Problem(A=A, b=np.ones(3), c=np.ones(2), cone=Cone(l=1, q=[0, 2]))   # SOC size 0
    with pytest.raises(sscs.SSCSError, match="invalid"):
        sscs.Solver(bad2)
    with pytest.raises(sscs.SSCSError, match="invalid"):
        sscs.Solver(Problem(A=A, b=np.ones(3), c=np.ones(2), cone=Cone(l=3)), sscs.Settings(mem=0))
    st = sscs.Settings()
    c = st.to_c()
    c.linsys = 7                                                             # no such linear step
    h = ctypes.c_void_p()
    mm = sscs._Marshal(A, np.ones(3), np.ones(2), Cone(l=3))
    assert sscs.lib().sscs_create(ctypes.byref(mm.data), ctypes.byref(mm.cone), ctypes.byref(c), None,
                                  ctypes.byref(h)) == -1


def test_noalloc_rejects_instances_beyond_its_scratch():
    # checked on the host before any device work: the 20000 x 50000 SOCP
    # (1e6 nonzeros) needs more than the 32 MiB static scratch
    from paper_1903_06477_amd import generators as G
    from paper_1903_06477_amd import sscs
    prob = G.config2_socp()
    with pytest.raises(sscs.SSCSError, match="32 MiB"):
        sscs.solve_noalloc(prob)
    bad = G.config1_lp()
    with pytest.raises(sscs.SSCSError, match="unsupported"):
        sscs.solve_noalloc(bad, sscs.Settings(precision="mixed"))
    with pytest.raises(sscs.SSCSError, match="unsupported"):
        sscs.solve_noalloc(bad, sscs.Settings(linsys="direct"))


def test_batch_create_rejects_unsupported_forms_on_the_host():
    # the batched engine's limits, checked before any device work: PSD blocks
    # above order 64, the mixed-precision form, the direct linear step
    import numpy as np
    from paper_1903_06477_amd import generators as G
    from paper_1903_06477_amd import sscs
    r = np.random.default_rng(0)
    cone = G.Cone(l=3, s=[65])
    m = cone.rows()
    psd65 = G.Problem(A=G.sprandn(m, 10, 0.05, r), b=r.standard_normal(m), c=r.standard_normal(10), cone=cone)
    with pytest.raises(sscs.SSCSError, match="unsupported"):
        sscs.BatchSolver([psd65])
    lp = G.config1_lp()
    with pytest.raises(sscs.SSCSError, match="unsupported"):
        sscs.BatchSolver([lp, lp], sscs.Settings(precision="mixed"))
    with pytest.raises(sscs.SSCSError, match="unsupported"):
        sscs.BatchSolver([lp, lp], sscs.Settings(linsys="direct"))
