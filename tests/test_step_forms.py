"""Host checks of the two rearrangements the FP32 step loop relies on (no GPU).

* Edge form: with z_m the midpoint of [z_j, z_(j+1)] and dz_m its width,
  dz_m sinc(phi dz_m / 2) e^(j phi z_m) = (e^(j phi z_(j+1)) - e^(j phi z_j)) / (j phi)
  (the exact integral of e^(j phi z) over the step), so the step sum of eq. (slow_vary) equals
  the sum of p_m times differences of edge phasors.
* Low-rank table: the scaled ODE profile ln rho(z_m, f_c) log2(e) / 2 of the O-to-U plan, as the
  oracle computes it, is within the kernel's bound of a rank-8 matrix, found by Gram-Schmidt
  with column pivoting; the FP32 forward relies on this to replace its per-step table reads.
* Projection on S (adjoint, FP32 form): with S = |S| e^(j theta),
  Re(conj(S) term_m) = |S| amp_m cos(phi z_m - theta) for a midpoint term amp_m e^(j phi z_m), and
  Re(conj(S) (e^(j phi z1) - e^(j phi z0)) / (j phi)) = |S| (sin(phi z1 - theta) - sin(phi z0 - theta)) / phi
  for an edge-form term; theta / (2 pi) comes from the kernel's FP32 atan_rev32, whose polynomial
  and octant logic are checked here against numpy's arctan2.
"""
import os
import re

import numpy as np

from oracle import oracle as O
from paper_2401_18022_amd import workloads as W


def _steps(M, L=80e3, alpha=4.6e-5):
    q = -np.expm1(-alpha * L)
    edge = -np.log1p(-q * np.arange(M + 1) / M) / alpha
    return edge, 0.5 * (edge[1:] + edge[:-1]), np.diff(edge)


def test_edge_form_equals_midpoint_sinc_form():
    rng = np.random.default_rng(11)
    edge, zm, dz = _steps(112)
    for phi in (3e-3, 5e-2, 1.0, 40.0, 1.4e3):   # rad/m: first step below and above |phi dz/2| = 1/2
        p = np.exp(rng.uniform(-4.0, 0.5, size=zm.size))
        mid = np.sum(p * dz * np.sinc(phi * dz / (2 * np.pi)) * np.exp(1j * phi * zm))
        e = np.exp(1j * phi * edge)
        edge_form = np.sum(p * (e[1:] - e[:-1])) / (1j * phi)
        assert abs(edge_form - mid) <= 1e-11 * np.sum(p * dz), phi


def _pivoted_gram_schmidt_residuals(L, terms):
    R = L.copy()
    out = [np.abs(R).max()]
    for _ in range(terms):
        j = int(np.argmax((R * R).sum(axis=0)))
        q = R[:, j] / np.linalg.norm(R[:, j])
        R -= np.outer(q, q @ R)
        out.append(np.abs(R).max())
    return np.array(out)


def test_ou_profile_table_is_rank_8_within_the_kernel_bound():
    wl = W.config_ou(grid_s=8, grid_v=8)
    ell = O.Oracle(wl.fibre, wl.plan).profile()["ell"]
    res = _pivoted_gram_schmidt_residuals(ell * (0.5 / np.log(2.0)), 8)
    assert res[8] <= 2.5e-7, res
    assert res[6] > 2.5e-7          # not trivially small: the first terms carry the profile
    assert np.all(np.diff(res) <= 0)


def test_projection_on_s_equals_re_conj_s_term():
    rng = np.random.default_rng(5)
    edge, zm, dz = _steps(112)
    for phi in (3e-3, 1.0, 1.4e3):
        p = np.exp(rng.uniform(-4.0, 0.5, size=zm.size))
        S = complex(*rng.normal(size=2)) * 1e3
        th = np.angle(S)
        tol = 1e-12 + 4e-16 * phi * edge[-1]  # FP64 rounding of phases up to phi L radians
        mid = p * dz * np.sinc(phi * dz / (2 * np.pi)) * np.exp(1j * phi * zm)
        amp = p * dz * np.sinc(phi * dz / (2 * np.pi))
        assert np.allclose((np.conj(S) * mid).real, abs(S) * amp * np.cos(phi * zm - th), rtol=0, atol=tol * abs(S) * amp.max())
        e = np.exp(1j * phi * edge)
        ed = p * (e[1:] - e[:-1]) / (1j * phi)
        sn = np.sin(phi * edge - th)
        proj = abs(S) * p * (sn[1:] - sn[:-1]) / phi
        assert np.allclose((np.conj(S) * ed).real, proj, rtol=0, atol=tol * abs(S) * p.max() * 2 / phi)


def _atan_rev32_coefficients():
    src = open(os.path.join(os.path.dirname(__file__), "..", "paper_2401_18022_amd", "csrc", "isrsgn_adjoint.hip")).read()
    body = src[src.index("__device__ inline float atan_rev32"):]
    body = body[:body.index("\n}\n")]
    first = float(re.search(r"float p = (-?[0-9.e-]+)f;", body).group(1))
    rest = [float(x) for x in re.findall(r"p = fmaf\(p, u, (-?[0-9.e-]+)f\);", body)]
    return [first] + rest  # highest degree first, Horner order


def _atan_rev32(y, x, coef):
    f = np.float32
    y, x = np.asarray(y, dtype=f), np.asarray(x, dtype=f)
    ax, ay = np.abs(x), np.abs(y)
    mx, mn = np.maximum(ax, ay), np.minimum(ax, ay)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(mx > 0, (mn / np.where(mx > 0, mx, f(1))).astype(f), f(0))
    u = (t * t).astype(f)
    p = np.full_like(t, f(coef[0]))
    for c in coef[1:]:
        p = (p * u + f(c)).astype(f)
    r = (p * t).astype(f)
    r = np.where(ay > ax, f(0.25) - r, r)
    r = np.where(x < 0, f(0.5) - r, r)
    return np.where(y < 0, -r, r)


def test_atan_rev32_matches_arctan2():
    coef = _atan_rev32_coefficients()
    assert len(coef) == 8
    rng = np.random.default_rng(3)
    y = rng.normal(size=200000) * 10.0 ** rng.uniform(-6, 6, size=200000)
    x = rng.normal(size=200000) * 10.0 ** rng.uniform(-6, 6, size=200000)
    y32, x32 = y.astype(np.float32), x.astype(np.float32)
    got = _atan_rev32(y32, x32, coef).astype(np.float64)
    ref = np.arctan2(y32.astype(np.float64), x32.astype(np.float64)) / (2 * np.pi)
    d = np.abs(got - ref)
    d = np.minimum(d, 1.0 - d)  # the phase is taken modulo one revolution
    assert d.max() < 5e-8, d.max()
    # axes and the origin: exact quarter turns, 0 for S = 0
    ax = _atan_rev32(np.array([0, 1, 0, -1, 0], np.float32), np.array([1, 0, -1, 0, 0], np.float32), coef)
    assert np.allclose(ax, [0.0, 0.25, 0.5, -0.25, 0.0], atol=1e-7)
