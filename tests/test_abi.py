"""Host-only checks of the C ABI (no device work): the library loads, exports
every symbol declared in include/slh.h, validates arguments before touching
the device, and reports footprints."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def S():
    from paper_2511_16821_amd import slh
    if not os.path.exists(slh.LIB_PATH):
        from paper_2511_16821_amd import build
        build.build()
    slh.lib()
    return slh


def _declared():
    txt = open(os.path.join(ROOT, "include", "slh.h")).read()
    return sorted(set(re.findall(r"\b(slh_[a-z_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported(S):
    L = S.lib()
    names = _declared()
    assert len(names) >= 19
    for n in names:
        assert hasattr(L, n), n
    assert sorted(S.EXPORTS) == names


def test_validation_rejects_before_allocating(S):
    import ctypes as C
    from paper_2511_16821_amd import workloads as W
    good = W.c1()
    bad_cases = [
        dict(nx=0), dict(dt=0.0), dict(dt=-1.0), dict(c=0.0), dict(n_s=-2),
        dict(sn_order=5), dict(sn_order=0), dict(n_particles=-5), dict(points=7),
        dict(precision=3), dict(w_cut_rel=-1.0), dict(x_hi=0.0),
        dict(n_s_cell=np.full(400, -2, dtype=np.int32)),
        dict(n_s_cell=np.full(400, 2_000_000, dtype=np.int32)),
        dict(boundary=16), dict(boundary=-1), dict(si_norm=2), dict(si_norm=-1),
        dict(steady_raw=2), dict(steady=True, horizon=-1.0),
        dict(steady=True, horizon=np.inf), dict(steady=True, horizon=1e16),
        dict(steady=True, w_cut_rel=0.0),  # the default horizon needs a cutoff
        dict(steady=True, sigma_a=np.where(np.arange(400) == 7, 0.0, 0.1)),
        dict(closure=2), dict(closure=-1), dict(si_accel=2), dict(si_accel=-1),
        dict(census_qmc=2), dict(census_qmc=-1),
        # an inflow on a reflective side, a non-finite inflow
        dict(boundary=1, inflow=np.where(np.arange(80) < 20, 1.0, 0.0)),
        dict(inflow=np.where(np.arange(80) == 50, np.nan, 0.0)),
        # census slots are 32-bit
        dict(census_cap=2 ** 31, n_particles=2 ** 31),
        # the diffusion correction needs sigma_t > 0 in steady state (a void)
        dict(si_accel=1, steady=True, horizon=50.0, sigma_a=np.where(np.arange(400) == 7, 0.0, 0.1),
             sigma_s=np.where(np.arange(400) == 7, 0.0, 1.0)),
        # the diffusion closure needs sigma_t > 0 in steady state (a void)
        dict(closure=1, steady=True, horizon=50.0, sigma_a=np.where(np.arange(400) == 7, 0.0, 0.1),
             sigma_s=np.where(np.arange(400) == 7, 0.0, 1.0)),
    ]
    for upd in bad_cases:
        p = dict(good)
        p.update({k: v for k, v in upd.items() if k not in ("nx", "steady_raw")})
        st, keep = S.make_problem(p)
        if "nx" in upd:
            st.nx = upd["nx"]
        if "steady_raw" in upd:
            st.steady = upd["steady_raw"]
        h = C.c_void_p()
        r = S.lib().slh_create(C.byref(st), None, S.ALLOC_FN(0), S.FREE_FN(0), None, C.byref(h))
        assert r == S.SLH_E_INVALID_ARG, upd
        assert not h.value
        assert S.lib().slh_last_error()
    for field, val in (("sigma_s", np.nan), ("sigma_a", -1.0), ("q", np.inf)):
        p = dict(good)
        arr = np.array(p[field], dtype=float)
        arr.flat[3] = val
        p[field] = arr
        st, keep = S.make_problem(p)
        h = C.c_void_p()
        r = S.lib().slh_create(C.byref(st), None, S.ALLOC_FN(0), S.FREE_FN(0), None, C.byref(h))
        assert r == S.SLH_E_INVALID_ARG, field
        assert b"finite" in S.lib().slh_last_error()


def test_footprint_scales_with_problem(S):
    from paper_2511_16821_amd import workloads as W
    # steady problems need no dt; voids are fine with an explicit horizon
    assert S.slh_footprint_bytes(W.duct()) > 0
    assert S.slh_footprint_bytes(W.slab_regions(dt=0.0)) > 0
    small = S.slh_footprint_bytes(W.c1())
    big = S.slh_footprint_bytes(W.c1(n_particles=10 ** 6))
    assert 0 < small < big
    p = W.c1()
    p["sn_order"] = 3
    assert S.slh_footprint_bytes(p) == 0


def test_null_arguments(S):
    import ctypes as C
    L = S.lib()
    assert L.slh_advance(None, 1) == S.SLH_E_INVALID_ARG
    assert L.slh_get_flux(None, 0, None) == S.SLH_E_INVALID_ARG
    assert L.slh_synchronize(None) == S.SLH_E_INVALID_ARG
    L.slh_destroy(None)
    assert L.slh_create(None, None, S.ALLOC_FN(0), S.FREE_FN(0), None,
                        C.byref(C.c_void_p())) == S.SLH_E_INVALID_ARG


def test_binding_matches_the_header(S):
    """The binding's constants and slh_problem field order are those the
    header declares (the ctypes struct mirrors the C layout field by field)."""
    txt = open(os.path.join(ROOT, "include", "slh.h")).read()
    for name, val in re.findall(r"#define (SLH_[A-Z0-9_]+) (\d+)u?\b", txt):
        if hasattr(S, name):
            assert getattr(S, name) == int(val), name
    for name in ("SLH_ABI_VERSION", "SLH_REFLECT_Y_HI", "SLH_SI_NORM_TOTAL", "SLH_CLOSE_DIFFUSION",
                 "SLH_ACCEL_DSA"):
        assert hasattr(S, name), name
    body = txt[txt.index("typedef struct {\n    uint32_t abi_version;"):txt.index("} slh_problem;")]
    fields = []
    for line in body.split("\n"):
        m = re.match(r"\s+(?:const\s+)?[a-z0-9_]+\s*\*?\s*([a-z_0-9, ]+);", line)
        if m:
            fields += [f.strip().lstrip("*") for f in m.group(1).split(",")]
    assert fields == [f for f, _ in S.slh_problem._fields_], fields
