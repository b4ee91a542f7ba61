"""Equal-time Green's function and log|det M| from the fields, stabilised by a
UDT (QR with column pivoting) chain.

The paper defines M = I + B_L ... B_1 and the weight through det M
(Determinant quantum Monte Carlo); it points to the standard DQMC literature
for how G = M^-1 is obtained without overflow.  This is the textbook
stabilisation: multiply the B's in blocks of n_stab slices, and after every
block re-factor the running product as U D T with a pivoted QR, so the huge
and tiny scales live only in the diagonal D.  At the end

    I + U D T = U Db (Db^-1 U^T + Ds T),   Db = max(D, 1), Ds = min(D, 1)
    G = (Db^-1 U^T + Ds T)^-1 Db^-1 U^T
    log|det M| = sum log Db + log|det(Db^-1 U^T + Ds T)|.

Parity: pinned by brute-force dense determinants / inverses of I + prod B at
small beta, by the g = 0, uniform-field and t = 0 closed forms, and by the
invariant that the rank-1-updated G of a sweep equals this recomputation
(tests/test_oracle_model.py, tests/test_oracle_sweep.py).
"""
import numpy as np
import scipy.linalg

from .model import b_matrix


def product_order(L, start):
    """Slices of the product B_{start-1} ... B_0 B_{L-1} ... B_start, rightmost first."""
    return [(start + j) % L for j in range(L)]


def block_product(p, expk, x, slices):
    """C = B_{slices[-1]} ... B_{slices[0]} by plain repeated multiplication."""
    c = b_matrix(p, expk, x[slices[0]])
    for l in slices[1:]:
        c = b_matrix(p, expk, x[l]) @ c
    return c


def udt_chain(p, expk, x, start):
    """U, D, T with U diag(D) T = B_{start-1} ... B_{start} (cyclic, all L slices)."""
    L, n, ns = p.L, p.n, p.n_stab
    if L % ns:
        raise ValueError("n_stab must divide L")
    order = product_order(L, start)
    U, D, T = np.eye(n), np.ones(n), np.eye(n)
    for b in range(L // ns):
        c = block_product(p, expk, x, order[b * ns:(b + 1) * ns])
        Z = (c @ U) * D[None, :]
        Q, R, piv = scipy.linalg.qr(Z, pivoting=True)
        D = np.abs(np.diag(R))
        rpt = np.empty_like(R)
        rpt[:, piv] = R                      # R P^T
        T = (rpt / D[:, None]) @ T
        U = Q
    return U, D, T


def green_from_udt(U, D, T):
    """G = (I + U D T)^-1 and log|det(I + U D T)| with the Db/Ds split."""
    db = np.maximum(D, 1.0)
    ds = np.minimum(D, 1.0)
    rhs = U.T / db[:, None]
    A = rhs + ds[:, None] * T
    G = np.linalg.solve(A, rhs)
    _, logabs = np.linalg.slogdet(A)
    return G, float(np.sum(np.log(db)) + logabs)


def green_and_logdet(p, expk, x, start=0):
    """G_{start-1} = (I + B_{start-1}...B_0 B_{L-1}...B_start)^-1 and log|det M|.

    With start = 0 this is G at the imaginary-time boundary, (I + B_{L-1}...B_0)^-1.
    log|det M| does not depend on start (cyclic invariance of the determinant).
    """
    return green_from_udt(*udt_chain(p, expk, x, start))
