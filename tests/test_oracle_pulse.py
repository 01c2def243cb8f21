"""Pins of the oracle pulse spectrum and synthesis against the paper's printed
values (Table 1, the epsilon column, the carrier index, the time origin)."""
import json
import os

import numpy as np
import pytest

from oracle import pulse, series
from workloads import Pulse, paper_sphere_pulse

GOLD = os.path.join(os.path.dirname(__file__), "golden")
W, T = 20.1, 128
DK = 2 * np.pi / W


def test_paper_pulse_spectrum_carrier_parity_and_ratios():
    g = json.load(open(os.path.join(GOLD, "paper_constants.json")))
    t1 = json.load(open(os.path.join(GOLD, "table1.json")))
    c = pulse.coefficients(paper_sphere_pulse(), 63, DK, T, 0.0)
    # odd pulse -> purely imaginary DFT
    assert np.max(np.abs(c.real)) < 1e-14 * np.max(np.abs(c))
    assert int(np.argmax(np.abs(c))) + 1 == g["carrier_index"]
    a = np.sort(np.abs(c))[::-1] / np.max(np.abs(c))
    for n, eps in zip(t1["n_terms"], t1["epsilon_lower_bound"]):
        # the n-th retained ratio, at the printed precision, reaches epsilon
        assert round(100 * a[n - 1], 1) >= round(100 * eps, 1)
    assert abs(a[4] - 0.2424) < 5e-4 and abs(a[9] - 0.0350) < 5e-4 and abs(a[19] - 0.0090) < 5e-4


def test_phase_factor_beta_matches_time_origin():
    # c_m with z_s = -(a + w/4) equals (DFT with index origin at tau = -4 pi N_c)
    # times e^{i beta}, beta = -k_m a [w/(4a) - 1]  (Sec. IV A)
    P = paper_sphere_pulse()
    c = pulse.coefficients(P, 63, DK, T, pulse.paper_time_shift(1.0, W))
    s = pulse.sample_points(W, T)
    F = pulse.pulse_samples(P, s)
    m = np.arange(1, 64)
    X = np.array([np.sum(F * np.exp(-2j * np.pi * mm * np.arange(T) / T)) for mm in m]) / T
    beta = -DK * m * (W / 4.0 - 1.0)
    assert np.max(np.abs(c - X * np.exp(1j * beta))) < 1e-15


def test_incident_reconstruction_and_time_origin():
    g = json.load(open(os.path.join(GOLD, "paper_constants.json")))
    P = paper_sphere_pulse()
    zs = pulse.paper_time_shift(1.0, W)
    c = pulse.coefficients(P, 63, DK, T, zs)
    # at sample-aligned positions the inverse DFT returns the shifted samples
    for j in (0, 5, 64, 100):
        z = zs + j * W / T
        xp = np.array([[0.0, 0.0, z]])
        p = pulse.synthesize(np.zeros((1, 63)), c, T, xp, DK, add_incident=True)[0]
        t = np.arange(T) * W / T
        s = z - t - zs
        s = (s + W / 2) % W - W / 2
        assert np.max(np.abs(p - pulse.pulse_samples(P, s))) < 1e-13
    # front at z = -a at t = 0; oscillation over the sphere until step 77 (1-based)
    tt = np.arange(T) * W / T
    back = (1.0 - tt - zs)          # travelling coordinate at z = +a
    on = np.abs(8 * np.pi * 1.0 / W * back) < 2 * np.pi * 1.0
    last = int(np.flatnonzero(on)[-1]) + 1
    assert last == g["last_step_oscillatory_on_sphere_1based"]
    front = (-1.0 - tt - zs)        # at z = -a
    assert abs(front[0] - W / 4) < 1e-12


def test_synthesis_equals_explicit_sum():
    rng = np.random.default_rng(1)
    U = rng.standard_normal((3, 16)) + 1j * rng.standard_normal((3, 16))
    c = rng.standard_normal(16) + 1j * rng.standard_normal(16)
    for TT in (32, 64):
        assert np.allclose(pulse.synthesize(U, c, TT), pulse.synthesize_direct(U, c, TT), atol=1e-12)


def test_table1_from_sphere_series():
    t1 = json.load(open(os.path.join(GOLD, "table1.json")))
    P = paper_sphere_pulse()
    c = pulse.coefficients(P, 63, DK, T, pulse.paper_time_shift(1.0, W))
    pts = np.array([[0.0, 0.0, -1.1], [0.0, 0.0, -4.0]])
    U = np.stack([series.scattered(DK * m, 1.0, "soft", pts) for m in range(1, 64)], axis=1)
    full = pulse.synthesize(U, c, T)
    for n, e11, e4 in zip(t1["n_terms"], t1["rms_percent_at_z_minus_1p1"], t1["rms_percent_at_z_minus_4"]):
        idx = pulse.dominant(c, n)
        ct = np.zeros_like(c)
        ct[idx] = c[idx]
        tr = pulse.synthesize(U, ct, T)
        assert abs(pulse.rms_error_percent(tr[0], full[0]) - e11) <= t1["printed_precision"] + 1e-9
        assert abs(pulse.rms_error_percent(tr[1], full[1]) - e4) <= t1["printed_precision"] + 1e-9


@pytest.mark.parametrize("kind,params", [("gauss", {"sigma": 0.8}), ("ricker", {"sigma": 1.1}),
                                         ("gsine", {"k0": 6.0, "sigma": 1.5})])
def test_smooth_pulse_coefficients_match_continuous_transform(kind, params):
    # For a smooth pulse well inside the period, c_m -> (1/L) * FT(k_m)
    dk, n_k, TT = 12.0 / 256, 256, 512
    L = 2 * np.pi / dk
    c = pulse.coefficients(Pulse(kind, params), n_k, dk, TT, 0.0)
    k = dk * np.arange(1, n_k + 1)
    if kind == "gauss":
        sg = params["sigma"]
        ft = sg * np.sqrt(2 * np.pi) * np.exp(-0.5 * (k * sg) ** 2)
    elif kind == "ricker":
        sg = params["sigma"]
        ft = sg ** 3 * np.sqrt(2 * np.pi) * k ** 2 * np.exp(-0.5 * (k * sg) ** 2)
    else:
        k0, sg = params["k0"], params["sigma"]
        a = lambda q: sg * np.sqrt(2 * np.pi) * np.exp(-0.5 * (q * sg) ** 2)
        ft = (a(k - k0) - a(k + k0)) / 2j
    assert np.max(np.abs(c - ft / L)) < 1e-12 * L


def test_table1_from_oracle_bem():
    """The oracle's own BEM (soft sphere, icosphere level 3, 642 nodes) in place
    of the series: the same truncated reconstructions land within the printed
    precision of Table 1 (Sec. IV A).  About 13 s of CPU."""
    from oracle import bie, field
    from oracle.mesh import Surface
    from workloads import Body, SOFT
    t1 = json.load(open(os.path.join(GOLD, "table1.json")))
    P = paper_sphere_pulse()
    c = pulse.coefficients(P, 63, DK, T, pulse.paper_time_shift(1.0, W))
    s = Surface([Body((0.0, 0.0, 0.0), 1.0, 1.0, 3, SOFT)])
    pts = np.array([[0.0, 0.0, -1.1], [0.0, 0.0, -4.0]])
    U = np.zeros((2, 63), dtype=np.complex128)
    for m in range(1, 64):
        phi, psi = bie.scatter_plane_wave(s, DK * m)
        U[:, m - 1] = field.field(s, DK * m, phi, psi, pts)[0]
    full = pulse.synthesize(U, c, T)
    for n, e11, e4 in zip(t1["n_terms"], t1["rms_percent_at_z_minus_1p1"], t1["rms_percent_at_z_minus_4"]):
        idx = pulse.dominant(c, n)
        ct = np.zeros_like(c)
        ct[idx] = c[idx]
        tr = pulse.synthesize(U, ct, T)
        assert abs(pulse.rms_error_percent(tr[0], full[0]) - e11) <= t1["printed_precision"] + 1e-9
        assert abs(pulse.rms_error_percent(tr[1], full[1]) - e4) <= t1["printed_precision"] + 1e-9


def _nwave_discrete_closed_form(sigma, dk, n_k, T):
    """c_m of the sampled N-wave F(s) = s / sigma on |s| <= sigma, from the
    closed form of the sum.  With h = L / T the samples are s = j h
    (j = -T/2 .. T/2 - 1), so c_m = (1/T) sum_{|j| <= J} (j h / sigma) e^{-i theta j},
    theta = k_m h, J = floor(sigma / h).  The sum is odd in j:
    sum_{|j|<=J} j e^{-i theta j} = -2i sum_{j=1}^{J} j sin(j theta), and
    sum_{j=1}^{J} j sin(j theta) = [(J+1) sin(J theta) - J sin((J+1) theta)] / (4 sin^2(theta/2))
    (minus the derivative of the Dirichlet kernel sum of cos(j theta))."""
    L = 2 * np.pi / dk
    h = L / T
    J = int(np.floor(sigma / h))
    assert J < T // 2
    th = dk * np.arange(1, n_k + 1) * h
    s = ((J + 1) * np.sin(J * th) - J * np.sin((J + 1) * th)) / (4.0 * np.sin(0.5 * th) ** 2)
    return (h / sigma) * (-2j) * s / T


def test_nwave_coefficients_closed_form_sum_and_continuous_limit():
    # window edge sigma/h = J + 0.37 (no sample on the jump, so no rounding
    # decides whether a sample is in the window)
    dk, n_k, T = 12.0 / 256, 256, 512
    h = 2 * np.pi / dk / T
    for J in (3, 11, 40):
        sigma = (J + 0.37) * h
        c = pulse.coefficients(Pulse("nwave", {"sigma": sigma}), n_k, dk, T, 0.0)
        ref = _nwave_discrete_closed_form(sigma, dk, n_k, T)
        assert np.max(np.abs(c - ref)) < 1e-13 * np.max(np.abs(ref))
    # continuous limit: the odd box-linear pulse has the transform
    # int_{-sigma}^{sigma} (s/sigma) e^{-iks} ds = (-2i/sigma)(sin(k sigma) - k sigma cos(k sigma))/k^2,
    # and the sampled sum approaches it at first order in h (the jumps at +-sigma)
    sigma = 1.1
    errs = []
    for TT in (1024, 2048, 4096, 8192):
        L = 2 * np.pi / dk
        c = pulse.coefficients(Pulse("nwave", {"sigma": sigma}), 64, dk, TT, 0.0)
        k = dk * np.arange(1, 65)
        ft = (-2j / sigma) * (np.sin(k * sigma) - k * sigma * np.cos(k * sigma)) / k ** 2
        errs.append(np.max(np.abs(c * L - ft)))
    errs = np.array(errs)
    hh = 2 * np.pi / dk / np.array([1024, 2048, 4096, 8192])
    assert np.all(errs <= 2.0 * hh)            # |jump| = 1 at each edge: error <= ~h
    assert errs[-1] < 0.5 * errs[0]            # and it shrinks with h (not monotonically:
    # the fractional position of the jumps on the grid changes with T)


@pytest.mark.parametrize("params", [{"ka": 3.0, "kb": 7.5, "D": 3.0},
                                    {"ka": 2.2, "kb": 8.8, "D": 2.1}, None])
def test_chirp_coefficients_match_complex_gaussian_integral(params):
    """The Gaussian-windowed linear chirp sin(ka s + (kb - ka) s^2 / (2D)) e^{-s^2/(2D^2)}
    is smooth and decays fast, so its sampled coefficients equal (1/L) times
    its continuous transform.  With sin = (e^{i phi} - e^{-i phi}) / 2i, each half
    is a complex Gaussian integral:
    int exp(-a s^2 + i b s) ds = sqrt(pi / a) exp(-b^2 / (4a)) for Re a > 0, with
    a = 1/(2D^2) -+ i beta, beta = (kb - ka)/(2D), b = +-ka - k."""
    if params is None:       # the seeded chirp of the space-time workload
        from workloads import spacetime_pulses
        params = [p for p in spacetime_pulses(0) if p.kind == "chirp"][0].params
    ka, kb, D = params["ka"], params["kb"], params["D"]
    dk, n_k, T = 12.0 / 256, 256, 2048
    L = 2 * np.pi / dk
    c = pulse.coefficients(Pulse("chirp", params), n_k, dk, T, 0.0)
    k = dk * np.arange(1, n_k + 1)
    beta = (kb - ka) / (2.0 * D)
    ap = 1.0 / (2 * D * D) - 1j * beta
    am = 1.0 / (2 * D * D) + 1j * beta
    plus = np.sqrt(np.pi / ap) * np.exp(-((ka - k) ** 2) / (4 * ap))
    minus = np.sqrt(np.pi / am) * np.exp(-((ka + k) ** 2) / (4 * am))
    ft = (plus - minus) / 2j
    assert np.max(np.abs(c - ft / L)) < 1e-12 * L
