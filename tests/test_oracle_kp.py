"""Pins of the oracle's SU(2) heat-bath draw (Kennedy-Pendleton) and of the
single-link update against the exact conditional density and a worked
example with the constant generator (Sec. 3.4 of the paper describes that
generator as its debugging tool)."""
import math

import numpy as np
import pytest
from scipy import integrate, special, stats

import oracle as O


def _a0_samples(alpha, n, seed, nhit=50):
    rng = np.random.default_rng(seed)
    out = []
    xs = []
    per = 4 * nhit + 2
    u = rng.random((n, per))
    for k in range(n):
        t, x, _ = O.kp_sample(alpha, nhit, u[k])
        if t >= 0:
            out.append(x[0])
            xs.append(x)
    return np.array(out), np.array(xs)


def kp_chi2_pvalue(a0, alpha, nb=40):
    """Chi^2 p-value of samples a0 against the exact density
    sqrt(1-a0^2) exp(alpha a0) / (pi I1(alpha)/alpha) on [-1, 1]."""
    norm = math.pi * special.iv(1, alpha) / alpha
    lo = max(-1.0, 1.0 - 12.0 / alpha) if alpha > 6 else -1.0
    edges = np.linspace(lo, 1.0, nb + 1)
    f = lambda a: math.sqrt(max(0.0, 1 - a * a)) * math.exp(alpha * a) / norm
    p = np.array([integrate.quad(f, edges[i], edges[i + 1])[0] for i in range(nb)])
    obs, _ = np.histogram(a0, bins=edges)
    n = len(a0)
    exp_c = np.append(p * n, (1.0 - p.sum()) * n)
    obs_c = np.append(obs, n - obs.sum())
    keep = exp_c > 5
    chi2 = (((obs_c[keep] - exp_c[keep]) ** 2) / exp_c[keep]).sum()
    dof = keep.sum() - 1
    return stats.chi2.sf(chi2, dof), chi2, dof


@pytest.mark.parametrize("alpha", [1.0, 3.0, 13.8])
def test_kp_a0_density_chi2(alpha):
    a0, _ = _a0_samples(alpha, 60000, seed=int(alpha * 10))
    # exact density sqrt(1-a0^2) exp(alpha a0), normalised by pi I1(alpha)/alpha
    norm = math.pi * special.iv(1, alpha) / alpha
    nb = 40
    lo = max(-1.0, 1.0 - 12.0 / alpha) if alpha > 6 else -1.0
    edges = np.linspace(lo, 1.0, nb + 1)
    f = lambda a: math.sqrt(max(0.0, 1 - a * a)) * math.exp(alpha * a) / norm
    p = np.array([integrate.quad(f, edges[i], edges[i + 1])[0] for i in range(nb)])
    p_out = 1.0 - p.sum()
    obs, _ = np.histogram(a0, bins=edges)
    n = len(a0)
    exp_c = np.append(p * n, p_out * n)
    obs_c = np.append(obs, n - obs.sum())
    keep = exp_c > 5
    chi2 = (((obs_c[keep] - exp_c[keep]) ** 2) / exp_c[keep]).sum()
    dof = keep.sum() - 1
    pval = stats.chi2.sf(chi2, dof)
    assert pval > 1e-4, (alpha, chi2, dof)


def test_kp_direction_isotropic():
    _, x = _a0_samples(3.0, 20000, seed=3)
    v = x[:, 1:]
    v = v / np.linalg.norm(v, axis=1)[:, None]
    n = len(v)
    assert np.all(np.abs(v.mean(axis=0)) < 5 / math.sqrt(3 * n))
    second = (v ** 2).mean(axis=0)
    assert np.all(np.abs(second - 1 / 3) < 5 * math.sqrt(4 / 45 / n))
    # unit quaternions
    assert np.abs(np.linalg.norm(x, axis=1) - 1).max() < 1e-14


def test_constant_generator_worked_example():
    # all uniforms 1/2: lambda^2 = ln2/alpha, accepted iff alpha >= (4/3) ln 2,
    # a0 = 1 - 2 ln2/alpha, direction cos(theta) = 0, phi = pi.
    for alpha in (13.8, 1.0):
        t, x, used = O.kp_sample(alpha, 10, np.full(42, 0.5))
        assert t == 0 and used == 6
        a0 = 1 - 2 * math.log(2) / alpha
        assert x[0] == pytest.approx(a0, abs=1e-15)
        assert x[1] == pytest.approx(-math.sqrt(1 - a0 * a0), abs=1e-15)
        assert abs(x[2]) < 1e-15 and abs(x[3]) < 1e-15
    t, x, used = O.kp_sample(0.9, 10, np.full(42, 0.5))  # 0.9 < (4/3) ln 2 = 0.924
    assert t == -1 and used == 40 and list(x) == [1, 0, 0, 0]


def test_first_cold_su2_update_constant_generator():
    # cold SU(2) lattice: staple = 6 * identity, so alpha = beta * 6 = 13.8 at
    # beta = 2.3, and the first updated link equals the KP draw x.
    L = O.Lattice(2, (4, 4, 4, 4), 2.3, rng=O.RNG_CONST, rng_const=0.5, start=O.COLD)
    A = L.staple(0, 0)
    assert np.allclose(A, 6 * np.eye(2), atol=1e-15)
    L.sweep(1, 0)
    links = L.get_links()
    a0 = 1 - 2 * math.log(2) / 13.8
    assert links[0, 0, 0] == pytest.approx(a0, abs=1e-13)
    assert links[0, 0, 1] == pytest.approx(-math.sqrt(1 - a0 * a0), abs=1e-13)


def test_single_link_heat_bath_conditional_density_su2():
    # For fixed staple A = k V, the heat bath samples U with density
    # exp(beta k Re Tr(U V)/2): x0 = Re Tr(U A)/(2k) has the KP density at
    # alpha = beta k (the SU(2) case of alpha = 2 beta k / N).
    rng = np.random.default_rng(17)
    beta = 2.0
    A = np.array([[1.3 + 0.4j, 0.2 - 0.7j], [-0.2 - 0.7j, 1.3 - 0.4j]])  # quaternion algebra element
    k = math.sqrt(abs(np.linalg.det(A)))
    alpha = beta * k
    U0 = np.array([1.0, 0, 0, 0])
    vals = []
    for s in range(30000):
        u = rng.random(4 * 10 + 2)
        out, used = O.update_link(2, beta, 10, 0, 0, U0, A, u)
        m = np.array([[out[0] + 1j * out[3], out[2] + 1j * out[1]],
                      [-out[2] + 1j * out[1], out[0] - 1j * out[3]]])
        if used != 40:  # accepted within NHIT tries (all ten rejected reads exactly 40)
            vals.append(0.5 * np.trace(m @ A).real / k)
    vals = np.array(vals)
    pval, chi2, dof = kp_chi2_pvalue(vals, alpha)
    assert pval > 1e-4, (chi2, dof)
    # a coupling off by a factor 2 (alpha = 2 beta k) is rejected by the same test
    assert kp_chi2_pvalue(vals, 2 * alpha)[0] < 1e-10


REJECT_TRY = [1e-300, 0.3, 1e-300, 1.0 - 2.0 ** -25]  # lambda^2 >> 1: a try that always fails


@pytest.mark.parametrize("g", [0, 1, 2])
def test_su3_subgroup_a0_density_chi2(g):
    """Cabibbo-Marinari: with the other two subgroups' single tries forced to
    fail, the SU(3) heat bath multiplies U by R = X V^dagger embedded in the
    rows/columns of subgroup g, where V = q/k is the normalised SU(2)
    projection of that block of M = U A; x0 = Re Tr(X)/2 must follow the KP
    density at alpha = (2 beta / 3) k."""
    rng = np.random.default_rng(40 + g)
    from helpers import haar_su
    a, b = [(0, 1), (1, 2), (0, 2)][g]
    c = 3 - a - b
    beta, nhit = 5.7, 1
    U = haar_su(3, 1, rng)[0]
    A = sum(haar_su(3, 6, rng))
    M = U @ A
    q = np.array([0.5 * (M[a, a] + M[b, b]).real, 0.5 * (M[a, b] + M[b, a]).imag,
                  0.5 * (M[a, b] - M[b, a]).real, 0.5 * (M[a, a] - M[b, b]).imag])
    k = float(np.linalg.norm(q))
    v = q / k
    V = np.array([[v[0] + 1j * v[3], v[2] + 1j * v[1]], [-v[2] + 1j * v[1], v[0] - 1j * v[3]]])
    alpha = 2.0 * beta * k / 3.0
    Uc = np.empty(18)
    Uc[0::2] = U.real.ravel()
    Uc[1::2] = U.imag.ravel()
    a0 = []
    for _ in range(40000):
        u = np.array(REJECT_TRY * g + list(rng.random(6)) + REJECT_TRY * (2 - g) + REJECT_TRY)
        out, used = O.update_link(3, beta, nhit, 0, 0, Uc, A, u)
        Un = (out[0::2] + 1j * out[1::2]).reshape(3, 3)
        R = Un @ U.conj().T
        # accepted in subgroup g only: R acts on rows/columns a, b alone
        if abs(R[c, c] - 1) > 1e-12 or abs(R[c, a]) + abs(R[c, b]) + abs(R[a, c]) + abs(R[b, c]) > 1e-12:
            continue
        if np.abs(R - np.eye(3)).max() < 1e-14:
            continue
        r = np.array([[R[a, a], R[a, b]], [R[b, a], R[b, b]]])
        X = r @ V
        a0.append(0.5 * np.trace(X).real)
    a0 = np.array(a0)
    assert len(a0) > 20000
    pval, chi2, dof = kp_chi2_pvalue(a0, alpha)
    assert pval > 1e-4, (g, alpha, chi2, dof)
    # a coupling with 1/2 in place of 1/N (the SU(2) normalisation) fails
    assert kp_chi2_pvalue(a0, beta * k)[0] < 1e-10


def test_su3_subgroup_heat_bath_preserves_unitarity():
    rng = np.random.default_rng(4)
    from helpers import haar_su, to_matrices, unitarity_error, det_error
    U = haar_su(3, 1, rng)[0]
    A = sum(haar_su(3, 6, rng))
    Uc = np.empty(18)
    Uc[0::2] = U.real.ravel()
    Uc[1::2] = U.imag.ravel()
    out, used = O.update_link(3, 5.7, 10, 0, 0, Uc, A, rng.random(3 * 42))
    m = to_matrices(out, 3)
    assert unitarity_error(m) < 1e-13 and det_error(m) < 1e-13
