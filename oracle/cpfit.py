"""O5: FP64 oracle for fitting CP factors to a tabular transition matrix
(test infrastructure; the GPU library never calls it).

Sec. 2.2 and Sec. 3 of the paper decompose the transition function into a
sum of rank-one terms but do not say how the terms are found.  The oracle
follows the standard alternating least squares of Kolda & Bader, "Tensor
Decompositions and Applications", SIAM Review 51(3), 2009, Sec. 3.4 (CP-ALS),
on the n-way tensor whose mode k pairs the current and next coordinate of
dimension k:
    X[u_0, .., u_{n-1}] = P(s' | s),   u_k = i_k m_k + j_k,
so that a rank-R model X ~ sum_r lambda_r a^(0)_r o .. o a^(n-1)_r is the CP
form P = sum_r lambda_r kron_k T^(k)_r with T^(k)_r = a^(k)_r reshaped m_k x m_k.
One ALS iteration visits k = 0 .. n-1 and sets
    A^(k) <- X_(k) (Khatri-Rao of the other factors) (Hadamard of their Grams)^+,
then scales every column of A^(k) to unit 2-norm, the norms becoming lambda.
The dense tensor is formed explicitly (tiny sizes); ``mttkrp_sparse`` is the
same product over COO entries for large sparse P.
"""
import numpy as np


def mode_sizes(sizes):
    return [int(m) * int(m) for m in sizes]


def dense_tensor(sizes, rows, cols, vals) -> np.ndarray:
    """X with X[u_0..u_{n-1}] = P[s, s'] (repeated (s, s') entries add up)."""
    sizes = [int(m) for m in sizes]
    X = np.zeros(mode_sizes(sizes))
    si = np.unravel_index(np.asarray(rows), sizes)
    sj = np.unravel_index(np.asarray(cols), sizes)
    idx = tuple(si[k] * sizes[k] + sj[k] for k in range(len(sizes)))
    np.add.at(X, idx, np.asarray(vals, np.float64))
    return X


def factors_from_flat(sizes, rank, flat):
    """[A^(0) .. A^(n-1)], A^(k) of shape (m_k^2, R), from the term layout of
    cpmdp_create (term r, dim k, m_k x m_k block row-major = index u_k)."""
    ms = mode_sizes(sizes)
    stride = sum(ms)
    flat = np.asarray(flat, np.float64)
    out, off = [], 0
    for mk in ms:
        out.append(np.stack([flat[r * stride + off: r * stride + off + mk] for r in range(rank)],
                            axis=1))
        off += mk
    return out


def factors_to_flat(A) -> np.ndarray:
    R = A[0].shape[1]
    return np.concatenate([np.concatenate([Ak[:, r] for Ak in A]) for r in range(R)])


def mttkrp(X, A, k):
    """M[u, r] = sum over every index with idx_k = u of X[idx] prod_{l != k} A^(l)[idx_l, r]
    (the matricised tensor times the Khatri-Rao product of the other factors),
    contracting one mode at a time."""
    n = X.ndim
    R = A[0].shape[1]
    M = np.zeros((X.shape[k], R))
    for r in range(R):
        Y = X
        for l in reversed(range(n)):
            if l != k:
                Y = np.tensordot(Y, A[l][:, r], axes=([l], [0]))
        M[:, r] = Y
    return M


def mttkrp_sparse(sizes, rows, cols, vals, A, k):
    """The same product over COO entries: each entry adds
    val * prod_{l != k} A^(l)[u_l, :] to row u_k."""
    sizes = [int(m) for m in sizes]
    si = np.unravel_index(np.asarray(rows), sizes)
    sj = np.unravel_index(np.asarray(cols), sizes)
    R = A[0].shape[1]
    prod = np.repeat(np.asarray(vals, np.float64)[:, None], R, axis=1)
    for l in range(len(sizes)):
        if l != k:
            prod *= A[l][si[l] * sizes[l] + sj[l], :]
    M = np.zeros((sizes[k] ** 2, R))
    np.add.at(M, si[k] * sizes[k] + sj[k], prod)
    return M


def reconstruct(A, lam) -> np.ndarray:
    """sum_r lambda_r a^(0)_r o .. o a^(n-1)_r as a dense tensor."""
    R = A[0].shape[1]
    X = np.zeros([Ak.shape[0] for Ak in A])
    for r in range(R):
        T = np.array(lam[r])
        for Ak in A:
            T = np.multiply.outer(T, Ak[:, r])
        X += T
    return X


def als(X, A0, iters):
    """CP-ALS (Kolda & Bader 2009, Sec. 3.4) from the factors A0 for a fixed
    number of iterations.  Returns (A, lambda, relative errors
    ||X - X_hat|| / ||X|| after every iteration, from the dense
    reconstruction)."""
    A = [np.array(Ak, np.float64) for Ak in A0]
    n = len(A)
    R = A[0].shape[1]
    lam = np.ones(R)
    normX = np.linalg.norm(X)
    errs = []
    for _ in range(iters):
        for k in range(n):
            V = np.ones((R, R))
            for l in range(n):
                if l != k:
                    V *= A[l].T @ A[l]
            Ak = mttkrp(X, A, k) @ np.linalg.pinv(V)
            lam = np.linalg.norm(Ak, axis=0)
            A[k] = Ak / np.where(lam > 0, lam, 1.0)
        errs.append(np.linalg.norm(X - reconstruct(A, lam)) / normX)
    return A, lam, np.asarray(errs)


def als_sparse(sizes, rows, cols, vals, A0, iters):
    """The same iterations as ``als`` with the Khatri-Rao product taken over
    COO entries (distinct (s, s') pairs), for P too large to form X.  The error comes from
    ||X - X_hat||^2 = ||X||^2 - 2 <X, X_hat> + ||X_hat||^2, with <X, X_hat> =
    sum_r lambda_r <M_r, a^(n-1)_r> (M of the last update, whose factor is
    the only one changed since) and ||X_hat||^2 = lambda^T (Hadamard of the
    Gram matrices) lambda."""
    A = [np.array(Ak, np.float64) for Ak in A0]
    n = len(A)
    R = A[0].shape[1]
    lam = np.ones(R)
    vals = np.asarray(vals, np.float64)
    normX2 = float(vals @ vals)
    errs = []
    for _ in range(iters):
        for k in range(n):
            V = np.ones((R, R))
            for l in range(n):
                if l != k:
                    V *= A[l].T @ A[l]
            M = mttkrp_sparse(sizes, rows, cols, vals, A, k)
            Ak = M @ np.linalg.pinv(V)
            lam = np.linalg.norm(Ak, axis=0)
            A[k] = Ak / np.where(lam > 0, lam, 1.0)
        inner = float(lam @ np.sum(M * A[n - 1], axis=0))
        H = np.ones((R, R))
        for Ak in A:
            H *= Ak.T @ Ak
        errs.append(np.sqrt(max(0.0, normX2 - 2 * inner + lam @ H @ lam)) / np.sqrt(normX2))
    return A, lam, np.asarray(errs)
