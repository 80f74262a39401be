"""CPU oracle for the LapH-subspace steps around the baryon block (test
infrastructure only: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it).

Sec. 2 of the paper writes the quark fields as combinations of Laplacian
eigenvectors (eq. (2)) and offers two routes to the block of eq. (3):

* reconstruct the fields from their coefficients (eq. (2)) and reduce over the
  lattice (eq. (3)) -- ``reconstruct`` here, then ``oracle.bblock``;
* precompute the spin-, noise- and flavour-blind mode triplets (eq. (4)) once
  and contract the coefficients onto them for every call -- ``mode_triplets``
  and ``mode_contract``.

Each function is the plain definition in complex128 (numpy matmul / einsum as
library primitives, no blocking).  Layouts follow the GPU boundary:

    phi  [V][3][n_ev]          phi[x][a][l] = phi^{(l)}_{a x}
    Q    [n_q][n_dil][n_ev]    Q[i][d][l]   = Q^{(d)}_{l} of coefficient set i
    q    [n_q][V][3][n_dil]    q[i][x][a][d] = q^{(d)}_{a x}
    T    [n_mom][n_ev][n_ev][n_ev]
    B    [n_mom][n1][n2][n3]
"""
from __future__ import annotations

import numpy as np


def reconstruct(Q, phi) -> np.ndarray:
    """eq. (2): q^{(d)}_{a x} = sum_l Q_{d l} phi^{(l)}_{a x}, for every
    coefficient set in Q ([n_q][n_dil][n_ev] or [n_dil][n_ev])."""
    phi = np.asarray(phi, dtype=np.complex128)
    Q = np.asarray(Q, dtype=np.complex128)
    if phi.ndim != 3 or phi.shape[1] != 3:
        raise ValueError("phi must have shape [V, 3, n_ev], got %r" % (phi.shape,))
    single = Q.ndim == 2
    Qs = Q[None] if single else Q
    if Qs.ndim != 3 or Qs.shape[2] != phi.shape[2]:
        raise ValueError("Q must have shape [n_q, n_dil, n_ev] with n_ev = %d" % phi.shape[2])
    V, n_ev = phi.shape[0], phi.shape[2]
    flat = phi.reshape(3 * V, n_ev)
    out = np.stack([(flat @ Qi.T).reshape(V, 3, Qi.shape[0]) for Qi in Qs])
    return out[0] if single else out


def mode_triplets(L: int, phi, mom) -> np.ndarray:
    """eq. (4): T^p_{l1 l2 l3} = sum_x exp(-i p.x) eps_abc phi^{(l1)}_{a x}
    phi^{(l2)}_{b x} phi^{(l3)}_{c x}.  This is eq. (3) with all three fields
    replaced by the eigenvectors, so it is the block oracle applied to phi."""
    import oracle
    return oracle.bblock(L, phi, phi, phi, mom)


def mode_contract(Q1, Q2, Q3, T) -> np.ndarray:
    """The baryon block from the mode triplets (Sec. 2, after eq. (4)):
    B^p_{d1 d2 d3} = sum_{l1 l2 l3} Q1_{d1 l1} Q2_{d2 l2} Q3_{d3 l3} T^p_{l1 l2 l3}."""
    Q1, Q2, Q3, T = (np.asarray(a, dtype=np.complex128) for a in (Q1, Q2, Q3, T))
    n_ev = T.shape[1]
    if T.ndim != 4 or T.shape[1:] != (n_ev, n_ev, n_ev):
        raise ValueError("T must have shape [n_mom, n_ev, n_ev, n_ev], got %r" % (T.shape,))
    for Qi in (Q1, Q2, Q3):
        if Qi.ndim != 2 or Qi.shape[1] != n_ev:
            raise ValueError("coefficients must have shape [n_dil, %d], got %r" % (n_ev, Qi.shape))
    return np.einsum("ai,bj,ck,pijk->pabc", Q1, Q2, Q3, T, optimize=True)
