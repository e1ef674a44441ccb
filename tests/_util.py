"""Shared helpers for the parity tests (comparison metrics only)."""
import numpy as np


def rel_errs(got, ref):
    """(normwise relative L2 error, max-abs error / max |ref|) of two arrays."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = got - ref
    nrm = float(np.linalg.norm(d) / max(np.linalg.norm(ref), 1e-300))
    mx = float(np.abs(d).max() / max(np.abs(ref).max(), 1e-300))
    return nrm, mx


def assert_close(got, ref, tol, what=""):
    nrm, mx = rel_errs(got, ref)
    assert nrm <= tol and mx <= tol, f"{what}: normwise {nrm:.3e}, max {mx:.3e} > {tol:.1e}"
    return nrm, mx


def ell_to_csr(idx, w, cnt, n_particles):
    """GPU ELL export ([K, n_nodes] slot-major) -> scipy CSR [n_nodes, N]."""
    import scipy.sparse as sp

    idx = np.asarray(idx)
    w = np.asarray(w)
    cnt = np.asarray(cnt)
    K, nn = idx.shape
    mask = np.arange(K)[:, None] < cnt[None, :]
    rows = np.broadcast_to(np.arange(nn)[None, :], (K, nn))[mask]
    M = sp.csr_matrix((w[mask], (rows, idx[mask])), shape=(nn, n_particles))
    M.sum_duplicates()
    return M
