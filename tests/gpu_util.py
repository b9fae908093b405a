"""Shared helpers for the GPU tests: move seeded inputs to the device and
compute the oracle side on the CPU."""
import numpy as np
import scipy.sparse as sp
import torch

from oracle import direct, pencil, spai
from paper_1606_01216_amd import airga
from synthetic import beam


def dev():
    return torch.device("cuda", 0)


def to_dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=dev(), dtype=dtype)


def set_pencil(ctx, pen):
    ctx.set_pencil(to_dev(pen.row_ptr, torch.int32), to_dev(pen.col_idx, torch.int32),
                   to_dev(pen.m_val, torch.float64), to_dev(pen.k_val, torch.float64),
                   pen.alpha, pen.beta)


def csr_of(pen, values):
    return pencil.csr(pen.n, pen.row_ptr, pen.col_idx, values)


def rel_err(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    nrm = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / nrm) if nrm > 0 else float(np.linalg.norm(x))


def reference(pen, shifts, f, precision="dd"):
    """Oracle X for every shift: array (nshift, m, n)."""
    return np.stack([direct.reference_solve(pen, s, f, precision) for s in shifts])


def grid_pencil(nx, ny, seed=0):
    """A 2-D 5-point pencil (rows of <= 5 entries, bandwidth nx): K = Laplacian
    with random positive conductances, M = lumped mass + small coupling. Used
    to exercise a pattern that is not the beam's."""
    rng = np.random.default_rng(seed)
    n = nx * ny
    idx = np.arange(n).reshape(ny, nx)
    rows, cols, kv, mv = [], [], [], []
    diag_k = np.zeros(n)
    diag_m = rng.uniform(1.0, 2.0, n)
    for (a, b) in ((idx[:, :-1], idx[:, 1:]), (idx[:-1, :], idx[1:, :])):
        a, b = a.ravel(), b.ravel()
        c = rng.uniform(0.5, 1.5, a.size)
        mc = rng.uniform(0.01, 0.05, a.size)
        for (i, j) in ((a, b), (b, a)):
            rows.append(i); cols.append(j); kv.append(-c); mv.append(mc)
        np.add.at(diag_k, a, c)
        np.add.at(diag_k, b, c)
    rows.append(np.arange(n)); cols.append(np.arange(n)); kv.append(diag_k + 0.01); mv.append(diag_m)
    r = np.concatenate(rows); c = np.concatenate(cols)
    K = sp.csr_matrix((np.concatenate(kv), (r, c)), shape=(n, n))
    M = sp.csr_matrix((np.concatenate(mv), (r, c)), shape=(n, n))
    K.sort_indices(); M.sort_indices()
    assert np.array_equal(K.indptr, M.indptr) and np.array_equal(K.indices, M.indices)
    return beam.Pencil(n=n, row_ptr=K.indptr.astype(np.int32), col_idx=K.indices.astype(np.int32),
                       m_val=M.data.copy(), k_val=K.data.copy())


__all__ = ["dev", "to_dev", "set_pencil", "csr_of", "rel_err", "reference", "grid_pencil",
           "airga", "beam", "direct", "pencil", "spai"]
