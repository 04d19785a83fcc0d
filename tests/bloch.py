"""Exact correlation functions of clean periodic lattices by Bloch sums
(test infrastructure, independent of the oracle and of the library).

For a lattice of L_a x L_b cells with orbitals ordered (a L_b + b) n_orb + o,
|k, o> = N_c^{-1/2} sum_R e^{i k.R} |R, o> diagonalises H into n_orb x n_orb
blocks H(k)_{oo'} = sum_d h_{oo'}(d) e^{i k.d}, so for any state psi0
C(t) = <psi0|e^{-iHt}|psi0> = sum_k sum_n |<u_nk|psi0(k)>|^2 e^{-i E_n(k) t}.
"""
import numpy as np


def graphene_hk(t, ka, kb):
    """H(k) of the paper's graphene cell, written from its hopping list:
    (0,0) 0->1, (1,0) 1->0, (0,1) 1->0, all equal to t, plus conjugates."""
    h10 = t * (1 + np.exp(1j * ka) + np.exp(1j * kb))   # <1|H|0>: d = 0, (1,0), (0,1)
    hk = np.zeros(ka.shape + (2, 2), dtype=np.complex128)
    hk[..., 1, 0] = h10
    hk[..., 0, 1] = np.conj(h10)
    return hk


def _k_grid(la, lb):
    ka = 2 * np.pi * np.arange(la)[:, None] / la * np.ones((1, lb))
    kb = 2 * np.pi * np.arange(lb)[None, :] / lb * np.ones((la, 1))
    return ka, kb


def _sum_over_levels(times, e, w, chunk=64):
    out = np.empty(len(times), dtype=np.complex128)
    for i in range(0, len(times), chunk):
        out[i:i + chunk] = np.exp(-1j * np.outer(times[i:i + chunk], e)) @ w
    return out


def corr_graphene(psi0, la, lb, t_hop, times):
    """C(t) of clean graphene (nearest-neighbour hopping t_hop) for the state psi0."""
    psi = psi0.reshape(la, lb, 2)
    ph = np.fft.fft2(psi, axes=(0, 1)) / np.sqrt(la * lb)    # <k,o|psi> up to the sign of k
    ka, kb = _k_grid(la, lb)
    e, u = np.linalg.eigh(graphene_hk(t_hop, ka, kb))
    w = np.abs(np.einsum("abon,abo->abn", u.conj(), ph)) ** 2
    return _sum_over_levels(np.asarray(times, dtype=np.float64), e.ravel(), w.ravel())


def corr_square(psi0, la, lb, t_hop, t2_hop, times):
    """C(t) of the clean square lattice with nearest (t_hop) and next-nearest
    (t2_hop) neighbour hopping: E(k) = 2t (cos ka + cos kb) + 4t' cos ka cos kb."""
    ph = np.fft.fft2(psi0.reshape(la, lb)) / np.sqrt(la * lb)
    ka, kb = _k_grid(la, lb)
    e = 2 * t_hop * (np.cos(ka) + np.cos(kb)) + 4 * t2_hop * np.cos(ka) * np.cos(kb)
    return _sum_over_levels(np.asarray(times, dtype=np.float64), e.ravel(), (np.abs(ph) ** 2).ravel())
