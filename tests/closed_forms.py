"""Closed forms the tests compare against, from the spectra of the model
matrices (no factorization involved): eigenvalues of the free-boundary path
and grid Laplacians, and the Schur complement of a dense border in the
Kronecker eigenbasis of the spatio-temporal field."""
import numpy as np

from paper_2609_29765_amd import workloads as W


def lam(m):
    """Eigenvalues of the free-boundary path Laplacian of m vertices."""
    return 2 - 2 * np.cos(np.pi * np.arange(m) / m)


def bordered_logdet(T, m, tau, kappa, rho, Bc, D):
    """logdet of [[tau kron(AR1, kappa^2 I + L), B], [B^T, D]] through the
    Kronecker eigenbasis and the Schur complement of the border."""
    av = np.linalg.eigvalsh(W.ar1_precision(T, rho).toarray())
    au, U = np.linalg.eigh(W.ar1_precision(T, rho).toarray())
    ev, V1 = np.linalg.eigh(W.path_laplacian(m).toarray())
    mu = kappa * kappa + ev[:, None] + ev[None, :]
    G = m * m
    ld_field = T * G * np.log(tau) + G * np.log(av).sum() + T * np.log(mu).sum()
    nb = Bc.shape[1]
    X = Bc.T.reshape(nb, T, m, m)
    Y = np.einsum("st,bsij,ip,jq->btpq", U, X, V1, V1, optimize=True)
    S = np.einsum("btpq,ctpq,t,pq->bc", Y, Y, 1.0 / au, 1.0 / mu, optimize=True) / tau
    sign, ld_s = np.linalg.slogdet(D - S)
    assert sign > 0
    return ld_field + ld_s
