"""Host checks of the two rearrangements the FP32 step loop relies on (no GPU).

* Edge form: with z_m the midpoint of [z_j, z_(j+1)] and dz_m its width,
  dz_m sinc(phi dz_m / 2) e^(j phi z_m) = (e^(j phi z_(j+1)) - e^(j phi z_j)) / (j phi)
  (the exact integral of e^(j phi z) over the step), so the step sum of eq. (slow_vary) equals
  the sum of p_m times differences of edge phasors.
* Low-rank table: the scaled ODE profile ln rho(z_m, f_c) log2(e) / 2 of the O-to-U plan, as the
  oracle computes it, is within the kernel's bound of a rank-8 matrix, found by Gram-Schmidt
  with column pivoting; the FP32 forward relies on this to replace its per-step table reads.
"""
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
