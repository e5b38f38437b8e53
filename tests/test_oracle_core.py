"""Pins of the oracle core against brute force, closed forms and textbook
identities (CPU only)."""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

from oracle import core
from oracle.core import Grid


def brute_dft(a, sign=-1):
    """prod-dimensional DFT as one dense sum over all index pairs."""
    shape = a.shape
    idx = np.indices(shape).reshape(len(shape), -1)      # (d, n)
    phase = np.zeros((idx.shape[1], idx.shape[1]))
    for d, N in enumerate(shape):
        phase += (np.outer(idx[d], idx[d]) % N) / N
    Wm = np.exp(sign * 2j * math.pi * phase)
    return (Wm @ a.reshape(-1)).reshape(shape)


@pytest.fixture(autouse=True)
def _restore_mode():
    m = core.get_dft_mode()
    yield
    core.set_dft_mode(m)


@pytest.mark.parametrize("shape", [(8, 8, 8), (6, 6, 6), (12, 12, 12), (8, 6), (4, 8, 6)])
@pytest.mark.parametrize("mode", ["naive", "library"])
def test_dft_matches_bruteforce(shape, mode):
    core.set_dft_mode(mode)
    rng = np.random.default_rng(1)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = brute_dft(a)
    scale = np.abs(ref).max()
    assert np.abs(core.fft(a) - ref).max() <= 1e-13 * scale
    refi = brute_dft(a, +1) / a.size
    assert np.abs(core.ifft_complex(a) - refi).max() <= 1e-13 * np.abs(refi).max()


@pytest.mark.parametrize("shape", [(16, 16, 16), (32, 24, 16), (64, 64)])
def test_dft_modes_agree_roundtrip_parseval(shape):
    rng = np.random.default_rng(2)
    a = rng.standard_normal(shape)
    core.set_dft_mode("naive")
    An = core.fft(a)
    core.set_dft_mode("library")
    Al = core.fft(a)
    assert np.abs(An - Al).max() <= 1e-13 * np.abs(Al).max()
    # Hermitian symmetry of a real input's spectrum
    flip = tuple(slice(None) for _ in shape)
    rev = np.conj(Al[tuple(np.s_[::-1] for _ in shape)])
    rev = np.roll(rev, 1, axis=tuple(range(len(shape))))
    assert np.abs(Al - rev).max() <= 1e-12 * np.abs(Al).max()
    assert np.abs(core.ifft(Al) - a).max() <= 1e-13
    assert abs(np.sum(np.abs(Al) ** 2) / a.size - np.sum(a * a)) <= 1e-12 * np.sum(a * a)
    del flip


def _grid3(n=16, X=(1.0, 1.5, math.pi)):
    return Grid((n, n + 8, n), X)


def test_spectral_derivatives_exact_on_trig_polynomials():
    g = _grid3()
    X, Y, Z = np.meshgrid(*[-Xd + (2 * Xd / N) * np.arange(N) for N, Xd in zip(g.n, g.half_len)],
                          indexing="ij")
    kx, ky, kz = [m * math.pi / Xd for m, Xd in zip((3, 5, 2), g.half_len)]
    f = np.sin(kx * X) * np.cos(ky * Y) * np.sin(kz * Z + 0.3)
    lap_exact = -(kx ** 2 + ky ** 2 + kz ** 2) * f
    assert np.abs(core.spectral_lap(f, g) - lap_exact).max() <= 1e-11 * np.abs(lap_exact).max()
    gx, gy, gz = core.spectral_grad(f, g)
    ex = kx * np.cos(kx * X) * np.cos(ky * Y) * np.sin(kz * Z + 0.3)
    ey = -ky * np.sin(kx * X) * np.sin(ky * Y) * np.sin(kz * Z + 0.3)
    ez = kz * np.sin(kx * X) * np.cos(ky * Y) * np.cos(kz * Z + 0.3)
    for a, b in ((gx, ex), (gy, ey), (gz, ez)):
        assert np.abs(a - b).max() <= 1e-11 * max(1.0, np.abs(b).max())
    # Nyquist mode (-1)^i along x: Laplacian eigenvalue -(pi N/(2X))^2, derivative zero
    nyq = np.cos(math.pi * np.arange(g.n[0]))[:, None, None] * np.ones(g.n)
    lam = (math.pi * g.n[0] / (2 * g.half_len[0])) ** 2
    assert np.abs(core.spectral_lap(nyq, g) + lam * nyq).max() <= 1e-10 * lam
    assert np.abs(core.spectral_grad(nyq, g)[0]).max() <= 1e-12


def test_lap_S_constant_g_is_textbook_laplacian():
    g = Grid((8, 12, 6), (1.0, 2.0, 0.5))
    idx = np.indices(g.n)
    for k in [(1, 2, 3), (4, 0, 1), (0, 6, 3)]:
        ph = sum(2 * math.pi * kd * idx[d] / g.n[d] for d, kd in enumerate(k))
        mode = np.cos(ph + 0.2)
        eig = -sum(4.0 / g.h[d] ** 2 * math.sin(math.pi * kd / g.n[d]) ** 2 for d, kd in enumerate(k))
        out = core.lap_S(mode, np.ones(g.n), g)
        assert np.abs(out - eig * mode).max() <= 1e-11 * abs(eig)
        assert np.abs(core.fd_symbol(g)[tuple(k)] + eig) <= 1e-11 * abs(eig)


def test_lap_S_kills_constants_symmetric_negative_semidefinite():
    rng = np.random.default_rng(3)
    g = Grid((10, 8, 6), (1.0, 1.0, 1.0))
    gg = 0.1 + rng.random(g.n)
    assert np.abs(core.lap_S(np.ones(g.n), gg, g)).max() <= 1e-12
    u, v = rng.standard_normal(g.n), rng.standard_normal(g.n)
    a = core.inner(core.lap_S(u, gg, g), v, g)
    b = core.inner(u, core.lap_S(v, gg, g), g)
    assert abs(a - b) <= 1e-12 * abs(a)
    assert core.inner(-core.lap_S(u, gg, g), u, g) >= 0.0


def _manufactured_lap_S(n):
    g = Grid((n, n), (math.pi, math.pi))
    x = -math.pi + g.h[0] * np.arange(n)
    X, Y = np.meshgrid(x, x, indexing="ij")
    u = np.sin(X) * np.cos(2 * Y)
    gg = 1.0 + 0.5 * np.sin(X + Y)
    ux, uy = np.cos(X) * np.cos(2 * Y), -2 * np.sin(X) * np.sin(2 * Y)
    gx = gy = 0.5 * np.cos(X + Y)
    exact = gx * ux + gy * uy + gg * (-u - 4 * u)
    return np.abs(core.lap_S(u, gg, g) - exact).max()


def test_lap_S_second_order_manufactured():
    e1, e2 = _manufactured_lap_S(32), _manufactured_lap_S(64)
    assert 3.8 <= e1 / e2 <= 4.2


def test_div_central_second_order():
    errs = []
    for n in (32, 64):
        g = Grid((n, n), (math.pi, math.pi))
        x = -math.pi + g.h[0] * np.arange(n)
        X, Y = np.meshgrid(x, x, indexing="ij")
        F = [np.sin(X) * np.cos(Y), np.cos(X + 2 * Y)]
        exact = np.cos(X) * np.cos(Y) - 2 * np.sin(X + 2 * Y)
        errs.append(np.abs(core.div_central(F, g) - exact).max())
    assert 3.8 <= errs[0] / errs[1] <= 4.2


def _dense_neg_lap(g):
    n = int(np.prod(g.n))
    eye = np.eye(n).reshape((n,) + g.n)
    return -core.lap_S(eye, np.ones(g.n), g).reshape(n, n).T


@pytest.mark.parametrize("shape", [(8, 8), (6, 8), (4, 6, 4)])
def test_lapinv_is_pseudo_inverse(shape):
    g = Grid(shape, tuple(1.0 + 0.25 * d for d in range(len(shape))))
    A = _dense_neg_lap(g)
    P = np.linalg.pinv(A)
    rng = np.random.default_rng(4)
    f = rng.standard_normal(shape)
    ref = (P @ f.reshape(-1)).reshape(shape)
    out = core.lapinv(f, g)
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()
    # -Delta_h (A f) = f - mean f
    assert np.abs(-core.lap_h(out, g) - (f - f.mean())).max() <= 1e-11
    # C: max absolute row sum of the dense pseudo-inverse
    C_dense = np.abs(P).sum(axis=1).max()
    assert abs(core.lapinv_inf_norm(g) - C_dense) <= 1e-12 * C_dense


@pytest.mark.parametrize("shape", [(8, 8), (6, 8, 4)])
def test_surface_band_inverse_full_band_special_cases(shape):
    """Band = whole grid: with g = 1 the band solve is the FFT-diagonalized
    pseudo-inverse (-Delta_h)^{-1}; with a variable g > 0 it inverts the
    operator:diff Delta_{S,h} of core.lap_S on mean-zero functions."""
    grid = Grid(shape, tuple(1.0 + 0.25 * d for d in range(len(shape))))
    rng = np.random.default_rng(11)
    f = rng.standard_normal(shape)
    full = np.ones(shape, dtype=bool)
    a = core.lapinv_S_band(f, np.ones(shape), full, grid)
    ref = core.lapinv(f, grid)
    assert np.abs(a - ref).max() <= 1e-11 * np.abs(ref).max()
    g = 0.05 + rng.random(shape)
    b = core.lapinv_S_band(f, g, full, grid)
    assert abs(b.mean()) <= 1e-13 * np.abs(b).max()
    assert np.abs(-core.lap_S(b, g, grid) - (f - f.mean())).max() <= 1e-10 * np.abs(f).max()


def _band_residual_loops(psi, f, g, mask, h):
    """Residual of the band problem by explicit loops over nodes and faces."""
    shape = mask.shape
    B = [i for i in np.ndindex(shape) if mask[i]]
    fm = sum(f[i] for i in B) / len(B)
    res = np.zeros(shape)
    for i in B:
        acc = 0.0
        for d in range(len(shape)):
            for step in (-1, 1):
                j = list(i)
                j[d] = (j[d] + step) % shape[d]
                j = tuple(j)
                if mask[j]:
                    acc += 0.5 * (g[i] + g[j]) * (psi[i] - psi[j]) / (h[d] * h[d])
        res[i] = acc - (f[i] - fm)
    return res, sum(psi[i] for i in B) / len(B)


def test_surface_band_inverse_on_a_shell_by_loops():
    """A connected shell band on a 10x9x8 grid with random g > 0: the loop
    residual of every band equation vanishes, the band mean of psi is 0, psi
    is 0 off the band, and the operator is symmetric on the band."""
    shape = (10, 9, 8)
    grid = Grid(shape, (1.0, 0.9, 0.8))
    X = np.meshgrid(*[np.arange(n) - (n - 1) / 2 for n in shape], indexing="ij")
    r = np.sqrt(sum(x * x for x in X))
    mask = (r > 1.6) & (r < 3.4)
    rng = np.random.default_rng(12)
    g = 1e-3 + rng.random(shape)
    f1, f2 = rng.standard_normal(shape), rng.standard_normal(shape)
    p1 = core.lapinv_S_band(f1, g, mask, grid)
    res, mean = _band_residual_loops(p1, f1, g, mask, grid.h)
    assert np.abs(res).max() <= 1e-9 * np.abs(f1).max() and abs(mean) <= 1e-13
    assert (p1[~mask] == 0).all()
    p2 = core.lapinv_S_band(f2, g, mask, grid)
    c1, c2 = f1 - f1[mask].mean(), f2 - f2[mask].mean()
    assert abs((p1 * c2)[mask].sum() - (c1 * p2)[mask].sum()) <= 1e-10 * abs((p1 * c2)[mask].sum())


def test_surface_band_inverse_norm():
    """C = ||(-Delta_S,h)^{-1}||_inf on a band: with g = 1 on the whole grid it
    is the circulant C of (-Delta_h)^{-1}; on a shell with variable g the
    dense X = A^+ (I - 11^T/nb) agrees column by column with the band solve
    applied to unit vectors."""
    grid = Grid((8, 8), (1.0, 1.25))
    full = np.ones((8, 8), dtype=bool)
    C = core.lapinv_S_band_inf_norm(np.ones((8, 8)), full, grid)
    assert abs(C - core.lapinv_inf_norm(grid)) <= 1e-12 * C
    shape = (12, 10)
    grid = Grid(shape, (1.0, 1.0))
    X = np.meshgrid(*[np.arange(n) - (n - 1) / 2 for n in shape], indexing="ij")
    r = np.sqrt(X[0] ** 2 + X[1] ** 2)
    mask = (r > 2.0) & (r < 4.2)
    g = 1e-3 + np.random.default_rng(13).random(shape)
    B = np.flatnonzero(mask.ravel())
    cols = []
    for j in B:
        e = np.zeros(mask.size)
        e[j] = 1.0
        cols.append(core.lapinv_S_band(e.reshape(shape), g, mask, grid).ravel()[B])
    Xs = np.array(cols).T
    C_cols = float(np.abs(Xs).sum(axis=1).max())
    C = core.lapinv_S_band_inf_norm(g, mask, grid)
    assert abs(C - C_cols) <= 1e-9 * C


def test_lapinv_norm_values():
    # values quoted for the 64^2 [-1,1)^2 and 128^3 [-1,1)^3 grids
    assert abs(core.lapinv_inf_norm(Grid((64, 64), (1.0, 1.0))) - 0.16784) < 5e-6


def _phi_ref(k, z):
    getcontext().prec = 60
    zd = Decimal(float(z))          # exact binary value of z
    e = (-zd).exp()
    if k == 0:
        return float(e)
    if k == 1:
        return float((1 - e) / zd)
    return float((e - 1 + zd) / (zd * zd))


def test_phi_functions_high_precision():
    zs = np.concatenate([np.logspace(-8, 3, 200), [0.0999999, 0.1, 0.1000001, 0.05, 0.2]])
    for k, fn in ((0, core.phi0), (1, core.phi1), (2, core.phi2)):
        zk = zs[zs < 700.0] if k == 0 else zs      # e^{-z} underflows FP64 beyond ~745
        got = fn(zk)
        ref = np.array([_phi_ref(k, float(z)) for z in zk])
        assert np.all(got > 0)
        assert np.max(np.abs(got - ref) / ref) <= 4e-15
    assert core.phi1(np.array([0.0]))[0] == 1.0 and core.phi2(np.array([0.0]))[0] == 0.5
    z = np.logspace(-6, 3, 50)
    assert np.allclose(core.phi1(z), (1 - core.phi0(z)) / z, rtol=1e-9)
    assert np.allclose(core.phi2(z), (1 - core.phi1(z)) / z, rtol=1e-6)


def test_nonlinearity_derivatives():
    s = np.linspace(-0.5, 1.5, 41)
    hstep = 1e-6
    assert np.allclose(core.Wp(s), (core.W(s + hstep) - core.W(s - hstep)) / (2 * hstep), atol=1e-6)
    assert np.allclose(core.Wpp(s), (core.Wp(s + hstep) - core.Wp(s - hstep)) / (2 * hstep), atol=1e-5)
    assert np.allclose(core.fp_ind(s), (core.f_ind(s + hstep) - core.f_ind(s - hstep)) / (2 * hstep), atol=1e-8)
    assert core.f_ind(0.0) == 0.0 and core.f_ind(1.0) == 1.0
    assert core.fp_ind(0.0) == 0.0 and core.fp_ind(1.0) == 0.0
    u = np.linspace(0, 1, 100001)
    assert abs(np.abs(core.Wpp(u)).max() - 36.0) < 1e-12
    assert abs(np.abs(6 - 12 * u).max() - 6.0) < 1e-12
    assert abs(core.fp_ind(u).max() - 1.5) < 1e-9
    assert abs(core.g_loc(u).max() - 9.0 / 8.0) < 1e-9
