"""Rewrites of CP instances as Tensor-Train and Tucker instances (test
helpers): the CP form is the special case of both, so the same operator
reached through either form pins the oracle and the library against the CP
path."""
import numpy as np

from paper_2103_00331_amd import instances as I


def cp_as_tt(inst) -> I.TTInstance:
    """Diagonal bonds: b_k = R_a inside, G_0[0, :, :, r] = lambda_r T^(0)_r,
    G_k[r, :, :, r] = T^(k)_r, G_{n-1}[r, :, :, 0] = T^(n-1)_r."""
    n, A = inst.n_dims, inst.n_actions
    sizes = [int(m) for m in inst.sizes]
    bonds = np.ones((A, n + 1), np.int32)
    blocks = []
    for a in range(A):
        terms = inst.terms_of(a)
        R = len(terms)
        if n > 1:
            bonds[a, 1:n] = R
        for k in range(n):
            m, bl, br = sizes[k], int(bonds[a, k]), int(bonds[a, k + 1])
            G = np.zeros((bl, m, m, br))
            for r, t in enumerate(terms):
                T = inst.factor(t, k) * (inst.lambdas[t] if k == 0 else 1.0)
                G[0 if bl == 1 else r, :, :, 0 if br == 1 else r] += T
            blocks.append(G.ravel())
    return I.TTInstance(np.asarray(sizes, np.int64), bonds, np.concatenate(blocks),
                        inst.rewards.copy(), inst.gamma, inst.terminal.copy(), inst.name + "_tt")


def cp_as_tucker(inst) -> I.TuckerInstance:
    """Superdiagonal core C[r, .., r] = lambda_r with U^(k)_r = T^(k)_r."""
    n, A = inst.n_dims, inst.n_actions
    cr = np.zeros((A, n), np.int32)
    cores, facs = [], []
    for a in range(A):
        terms = inst.terms_of(a)
        R = len(terms)
        cr[a] = R
        C = np.zeros((R,) * n)
        for r, t in enumerate(terms):
            C[(r,) * n] = inst.lambdas[t]
        cores.append(C.ravel())
        for k in range(n):
            for t in terms:
                facs.append(inst.factor(t, k).ravel())
    return I.TuckerInstance(inst.sizes.copy(), cr, np.concatenate(cores), np.concatenate(facs),
                            inst.rewards.copy(), inst.gamma, inst.terminal.copy(),
                            inst.name + "_tucker")


def mixture_move_tt(sizes, p: float, gamma: float = 0.9, seed: int = 0) -> I.TTInstance:
    """Two dims, one action: with probability p a clamped +1 move along dim 0,
    else a clamped +1 move along dim 1, written with a bond of 2 (bond 0
    carries the dim-0 move, bond 1 the dim-1 move)."""
    m0, m1 = sizes
    S0, S1 = I.shift_matrix(m0, 1), I.shift_matrix(m1, 1)
    G0 = np.zeros((1, m0, m0, 2))
    G0[0, :, :, 0] = p * S0
    G0[0, :, :, 1] = (1 - p) * np.eye(m0)
    G1 = np.zeros((2, m1, m1, 1))
    G1[0, :, :, 0] = np.eye(m1)
    G1[1, :, :, 0] = S1
    rng = np.random.default_rng(seed)
    S = m0 * m1
    return I.TTInstance(np.asarray(sizes, np.int64), np.array([[1, 2, 1]], np.int32),
                        np.concatenate([G0.ravel(), G1.ravel()]), rng.normal(0, 1, S), gamma,
                        np.zeros(S, np.uint8), "mixture_move")
