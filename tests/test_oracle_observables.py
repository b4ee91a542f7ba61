"""Pins of the oracle's equal-time observables by exact many-body traces.

For a fixed phonon field the fermions are free, and the equal-time
expectation of any operator O at the imaginary-time boundary is

    <O>_x = Tr[B_{L-1} ... B_0 O] / Tr[B_{L-1} ... B_0]

with B_l the many-body operator exp(-dtau sum_s g x_l . n_s) exp(-dtau sum_s c_s^+ K c_s)
(paper: Determinant quantum Monte Carlo, the trace over the fermions).  Here
those operators are built as dense matrices over the full Fock space of both
spins on a 2x2 lattice (8 modes, 256 states, Jordan-Wigner signs), so
nothing of Wick's theorem, of the spin factors or of the determinant formula
enters the expected values.  The oracle's G, log|det M| and its density
correlations, double occupancy, density and S_CDW(pi, pi) are compared with
the traces.  A transposed G in the exchange term, a wrong spin factor or a
same-spin product in place of the cross-spin one fails here.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import dqmc, model, udt
from oracle.model import Params


def fock_annihilators(modes):
    """Dense c_m over 2^modes occupation states, state bit m = occupation of
    mode m, c_m |s> = (-1)^(number of occupied modes below m) |s - e_m>."""
    dim = 1 << modes
    ops = []
    for m in range(modes):
        c = np.zeros((dim, dim))
        for s in range(dim):
            if (s >> m) & 1:
                sign = -1.0 if bin(s & ((1 << m) - 1)).count("1") % 2 else 1.0
                c[s ^ (1 << m), s] = sign
        ops.append(c)
    return ops


def many_body_weights(p, x):
    """The 256 x 256 matrix B_{L-1} ... B_0 of both spins (modes i + N s)."""
    n = p.n
    c = fock_annihilators(2 * n)
    cd = [op.T for op in c]
    num = [cd[m] @ c[m] for m in range(2 * n)]
    K = model.hopping_matrix(p)
    hk = np.zeros_like(num[0])
    for s in range(2):
        for i in range(n):
            for j in range(n):
                if K[i, j] != 0.0:
                    hk += K[i, j] * (cd[i + n * s] @ c[j + n * s])
    ek = scipy.linalg.expm(-p.dtau * hk)
    A = np.eye(1 << (2 * n))
    for l in range(p.L):
        hv = sum(p.g * x[l, i] * (num[i] + num[i + n]) for i in range(n))
        bl = np.diag(np.exp(-p.dtau * np.diag(hv))) @ ek   # hv is diagonal in occupations
        A = bl @ A
    return A, c, cd, num


CASES = [
    Params(nx=2, t=1.0, mu=0.3, g=1.0, beta=1.0, dtau=0.25, n_stab=2),
    Params(nx=2, t=0.7, mu=-0.4, g=1.4, beta=1.2, dtau=0.2, n_stab=3),
]


@pytest.mark.parametrize("p", CASES)
def test_observables_match_fock_space_traces(p):
    rng = np.random.default_rng(11)
    x = 1.3 * rng.standard_normal((p.L, p.n))
    A, c, cd, num = many_body_weights(p, x)
    Z = np.trace(A)
    n = p.n

    def expect(op):
        return float(np.trace(A @ op) / Z)

    expk = model.exp_hopping(p, -1.0)
    G, logdet = udt.green_and_logdet(p, expk, x, 0)
    assert not np.allclose(G, G.T, atol=1e-3), "a symmetric G would not test the exchange term's index order"

    # Tr over both spins = det(I + B_{L-1}...B_0)^2
    assert abs(np.log(Z) - 2.0 * logdet) < 1e-11 * max(1.0, abs(np.log(Z)))
    # G_ij = <c_i c_j^+> for either spin
    for s in range(2):
        Gfock = np.array([[expect(c[i + n * s] @ cd[j + n * s]) for j in range(n)] for i in range(n)])
        assert np.max(np.abs(Gfock - G)) < 1e-12

    dens = [num[i] + num[i + n] for i in range(n)]
    nn_fock = np.array([[expect(dens[i] @ dens[j]) for j in range(n)] for i in range(n)])
    nn = dqmc.density_correlations(G)
    assert np.max(np.abs(nn - nn_fock)) < 1e-11

    obs = dqmc.equal_time_observables(p, G, x)
    eps = np.array([(-1.0) ** ((i % p.nx) + (i // p.nx)) for i in range(n)])
    s_cdw = float(eps @ nn_fock @ eps) / n
    docc = sum(expect(num[i] @ num[i + n]) for i in range(n)) / n
    density = sum(expect(dens[i]) for i in range(n)) / n
    assert abs(obs["s_cdw"] - s_cdw) < 1e-11
    assert abs(obs["double_occupancy"] - docc) < 1e-12
    assert abs(obs["density"] - density) < 1e-12
    # the cases are away from half filling and from the atomic limit: the
    # correlations are not products of densities
    assert abs(docc - (density / 2) ** 2) > 1e-4


def test_fock_annihilators_anticommute():
    """The Jordan-Wigner operators are fermionic: {c_a, c_b^+} = delta_ab, {c_a, c_b} = 0."""
    c = fock_annihilators(4)
    eye = np.eye(16)
    for a in range(4):
        for b in range(4):
            assert np.array_equal(c[a] @ c[b].T + c[b].T @ c[a], eye if a == b else 0 * eye)
            assert not np.any(c[a] @ c[b] + c[b] @ c[a])
