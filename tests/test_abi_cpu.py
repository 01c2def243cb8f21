"""CPU checks of the C ABI: the library loads, exports every declared entry
point, and its host-only parts (mesh builder, pulse coefficients, argument
checks) agree with the oracle.  No GPU work is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import mesh as omesh
from oracle import pulse as opulse
from workloads import Body, Pulse, uneven_bodies_workload, paper_sphere_pulse

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bem.h")

native = pytest.importorskip("paper_1706_07919_amd.native")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(native.LIB_PATH):
        pytest.fail("libbem.so is not built (run __graft_entry__.build())")
    return native.load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:bem_status|void|int32_t|const char\*)\s+(\w+)\s*\(", src, flags=re.M)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 15
    raw = ctypes.CDLL(native.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), n
    assert set(names) == set(native.EXPORTED)


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_mesh_bit_exact_vs_oracle_sphere(lib, level):
    body = Body((0.0, 0.0, -1.85), 1.0, 1.0, level, 0)
    x, n, w, f = native.bem_mesh_icosphere(level, 1.0, 1.0, (0.0, 0.0, -1.85), True)
    ox, on, ow, of = omesh.body_surface(body, True)
    assert np.array_equal(f, of)
    assert x.tobytes() == ox.tobytes()
    assert n.tobytes() == on.tobytes()
    assert w.tobytes() == ow.tobytes()


def test_mesh_bit_exact_vs_oracle_uneven_bodies(lib):
    for body in uneven_bodies_workload().bodies:
        if body.level > 4:
            continue
        for rescale in (True, False):
            x, n, w, f = native.bem_mesh_icosphere(body.level, body.radius, body.aspect,
                                                   body.center, rescale)
            ox, on, ow, of = omesh.body_surface(body, rescale)
            assert x.tobytes() == ox.tobytes() and n.tobytes() == on.tobytes()
            assert w.tobytes() == ow.tobytes() and np.array_equal(f, of)


def test_mesh_counts_and_invalid(lib):
    assert native.bem_mesh_counts(4) == (2562, 5120)
    with pytest.raises(native.BemError):
        native.bem_mesh_icosphere(2, -1.0, 1.0, (0, 0, 0))
    with pytest.raises(native.BemError):
        native.bem_mesh_icosphere(2, 1.0, 0.5, (0, 0, 0))
    with pytest.raises(native.BemError):
        native.bem_mesh_counts(9)


@pytest.mark.parametrize("pulse,dk,n_k,T,zs", [
    (paper_sphere_pulse(), 2 * np.pi / 20.1, 63, 128, -(1.0 + 20.1 / 4)),
    (Pulse("gauss", {"sigma": 0.7}), 12.0 / 64, 64, 128, -12.0),
    (Pulse("ricker", {"sigma": 1.2}), 12.0 / 64, 64, 256, -3.0),
    (Pulse("nwave", {"sigma": 0.9}), 12.0 / 64, 64, 128, 0.0),
    (Pulse("chirp", {"ka": 3.0, "kb": 7.5, "D": 2.5}), 12.0 / 64, 64, 128, -12.0),
    (Pulse("gsine", {"k0": 6.0, "sigma": 1.5}), 12.0 / 64, 64, 128, -12.0),
    (Pulse("gaussk", {"k0": 3.0, "width": 1.0}), 6.0 / 32, 32, 64, 0.0),
])
def test_pulse_coefficients_vs_oracle(lib, pulse, dk, n_k, T, zs):
    order = {"paper": ("Nc", "alpha", "w"), "gauss": ("sigma",), "ricker": ("sigma",),
             "nwave": ("sigma",), "chirp": ("ka", "kb", "D"), "gsine": ("k0", "sigma"),
             "gaussk": ("k0", "width")}[pulse.kind]
    params = [pulse.params[k] for k in order]
    got = native.bem_pulse_coeffs(pulse.kind, params, dk, n_k, T, zs)
    ref = opulse.coefficients(pulse, n_k, dk, T, zs)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_pulse_coefficients_invalid(lib):
    with pytest.raises(native.BemError):
        native.bem_pulse_coeffs("gauss", [0.5], -1.0, 8, 64, 0.0)
    with pytest.raises(native.BemError):
        native.bem_pulse_coeffs(9, [0.5], 1.0, 8, 64, 0.0)


def test_dominant_selection_matches_oracle(lib):
    c = opulse.coefficients(paper_sphere_pulse(), 63, 2 * np.pi / 20.1, 128, -(1.0 + 20.1 / 4))
    for n in (1, 5, 10, 20, 63):
        got = native.bem_pulse_dominant(c, n)
        assert np.array_equal(got, opulse.dominant(c, n) + 1)
    # equal magnitudes rank by lower index
    tie = np.array([0.5, 1.0, 1j, -1.0, 0.25 + 0j, -1j])
    assert list(native.bem_pulse_dominant(tie, 2)) == [2, 3]
    assert list(native.bem_pulse_dominant(tie, 4)) == [2, 3, 4, 6]
    assert np.array_equal(native.bem_pulse_dominant(tie, 3), opulse.dominant(tie, 3) + 1)
    rng = np.random.default_rng(3)
    r = rng.standard_normal(200) + 1j * rng.standard_normal(200)
    assert np.array_equal(native.bem_pulse_dominant(r, 37), opulse.dominant(r, 37) + 1)


def test_dominant_selection_invalid(lib):
    with pytest.raises(native.BemError):
        native.bem_pulse_dominant(np.ones(4, complex), 5)
    with pytest.raises(native.BemError):
        native.bem_pulse_dominant(np.ones(4, complex), 0)
    with pytest.raises(native.BemError):
        native.bem_pulse_dominant(np.array([1.0, np.nan]), 1)


@pytest.mark.parametrize("nt,nph,radius,tilt,center", [
    (2, 3, 1.0, 0.0, (0.0, 0.0, 0.0)),
    (12, 16, 1.0, 0.15 * np.pi, (0.1, -0.2, 0.3)),
    (48, 96, 1.3, 0.47, (1.0, 2.0, -3.0)),
])
def test_bowl_mesh_bit_exact_vs_oracle(lib, nt, nph, radius, tilt, center):
    got = native.bem_mesh_bowl(nt, nph, radius, tilt, center)
    ref = omesh.bowl(nt, nph, radius, tilt, center)
    for g, r in zip(got, ref):
        assert np.array_equal(g, r)


def test_bowl_mesh_invalid(lib):
    for args in [(1, 8), (8, 2)]:
        with pytest.raises(native.BemError):
            native.bem_mesh_bowl(*args)
    with pytest.raises(native.BemError):
        native.bem_mesh_bowl(8, 8, radius=-1.0)


@pytest.mark.parametrize("nu,radius,aspect,center", [(1, 1.0, 1.0, (0.0, 0.0, 0.0)),
                                                     (2, 0.7, 1.8, (0.3, -1.0, 2.0)),
                                                     (5, 1.0, 1.0, (0.0, 0.0, 0.0))])
def test_quadratic_mesh_bit_exact_vs_oracle(nu, radius, aspect, center):
    """The library's six-node geodesic mesh (host builder) equals the oracle's
    bit for bit: node coordinates, normals and the element table; nu = 5 is the
    paper's 500-element, 1002-node sphere."""
    from oracle.quadratic import QuadSurface
    from workloads import Body, HARD
    x, nrm, elems = native.bem_mesh_quadratic(nu, radius, aspect, center)
    qs = QuadSurface(Body(center, radius, aspect, 0, HARD), nu)
    assert x.shape == qs.x.shape and elems.shape == qs.elems.shape
    assert np.array_equal(elems, qs.elems)
    assert np.array_equal(x.view(np.uint64), qs.x.view(np.uint64))
    assert np.array_equal(nrm.view(np.uint64), qs.nrm.view(np.uint64))
    with pytest.raises(native.BemError):
        native.bem_mesh_quadratic(0)
