"""CPU checks of the inclusion study's analytic parts (Sec. 4.3)."""
import numpy as np

from paper_2605_09097_amd import eshelby


def test_pressure_closed_form():
    # Equal materials: P = delta / (1/(2G) + (1 - 2 nu)/(2G)) = delta G / (1 - nu)
    E, nu, d = 1e5, 0.3, 0.01
    G = E / (2 * (1 + nu))
    assert abs(eshelby.contact_pressure(d, E, E, nu, nu) - d * G / (1 - nu)) < 1e-9
    # A rigid inclusion loads the matrix by its own compliance alone: P -> 2 G_out delta
    assert abs(eshelby.contact_pressure(d, E, 1e12, nu, nu) - 2 * G * d) < 1e-3


def test_exact_field_traction_continuity_and_equilibrium():
    R, Pc = 0.05, 641.0
    # inside: hydrostatic; the radial traction is continuous at r = R
    xi = np.array([[0.5 + 0.3 * R, 0.5 + 0.2 * R]])
    assert np.allclose(eshelby.exact_stress(xi, R, Pc)[0], -Pc * np.eye(2))
    th = 0.7
    e = np.array([np.cos(th), np.sin(th)])
    out = eshelby.exact_stress(np.array([[0.5, 0.5]]) + (R * (1 + 1e-12)) * e, R, Pc)[0]
    assert abs(e @ out @ e + Pc) < 1e-6 * Pc
    # outside: divergence-free (central differences of the Cartesian field)
    h = 1e-6
    x0 = np.array([0.62, 0.57])
    div = np.zeros(2)
    for a in range(2):
        dp = np.zeros(2)
        dp[a] = h
        sp = eshelby.exact_stress(np.array([x0 + dp]), R, Pc)[0]
        sm = eshelby.exact_stress(np.array([x0 - dp]), R, Pc)[0]
        div += (sp[:, a] - sm[:, a]) / (2 * h)
    assert np.abs(div).max() < 1e-6 * Pc / R


def test_cauchy_stress_limits():
    mu, lam = eshelby.lame(np.array([1e5]), np.array([0.3]))
    assert np.allclose(eshelby.cauchy_stress(np.eye(2)[None], mu, lam), 0.0)
    # small uniform dilation: linear plane-strain response 2 (mu + lam) eps I
    eps = 1e-7
    s = eshelby.cauchy_stress(((1 + eps) * np.eye(2))[None], mu, lam)[0]
    assert np.allclose(s, 2 * (mu[0] + lam[0]) * eps * np.eye(2), rtol=1e-5)
