"""Seeded synthetic inputs: a clamped Euler-Bernoulli cantilever discretised with
Hermite-cubic beam elements, plus load vectors and shift lists.

This module only *produces inputs*: the mass and stiffness matrices M and K of
the second-order system of eq. (1.1) (M x'' + D x' + K x = F u with proportional
damping D = alpha M + beta K), the input matrix F and the expansion points.
It holds none of the method's arithmetic (no shifted operator, no
preconditioner, no Krylov solver); both the CPU oracle and the HIP library
consume exactly the arrays built here.

The paper's own beam matrices (the 1-D beam of its Section 5) are not
available; the element matrices below are the textbook Hermite-cubic
Euler-Bernoulli element (two DOFs per node: deflection w and rotation theta).

Layout conventions (shared with every consumer):
  * DOF order per node is (w_i, theta_i); node 0 is clamped and removed, so a
    beam of ``n_el`` elements has n = 2 * n_el DOFs and the tip deflection is
    DOF n - 2.
  * M and K share ONE structural CSR pattern (0-based int32 ``row_ptr``,
    ``col_idx`` with sorted columns): the 2x2-block tridiagonal node coupling,
    nnz = 6n - 8, with explicit zeros kept where contributions cancel.
  * F is stored as an (m, n) C-contiguous float64 array, i.e. an n x m
    column-major matrix with leading dimension n.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Damping coefficients D = ALPHA*M + BETA*K used by every workload (both lie in
# (0, 1) as the paper's experiments require).
ALPHA = 0.01
BETA = 0.001


@dataclasses.dataclass
class Pencil:
    """The sparse pencil (M, K) on one shared structural pattern."""

    n: int
    row_ptr: np.ndarray  # int32, n+1
    col_idx: np.ndarray  # int32, nnz
    m_val: np.ndarray    # float64, nnz
    k_val: np.ndarray    # float64, nnz
    alpha: float = ALPHA
    beta: float = BETA
    ei: np.ndarray | None = None  # per-element bending stiffness actually used

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])


def element_matrices(h: float):
    """Hermite-cubic beam element for unit EI and unit rhoA: (k_e, m_e), 4x4.

    Local DOFs are (w_a, theta_a, w_b, theta_b); k_e scales with EI / h^3,
    m_e with rhoA * h / 420.
    """
    k = np.array(
        [[12.0, 6.0 * h, -12.0, 6.0 * h],
         [6.0 * h, 4.0 * h * h, -6.0 * h, 2.0 * h * h],
         [-12.0, -6.0 * h, 12.0, -6.0 * h],
         [6.0 * h, 2.0 * h * h, -6.0 * h, 4.0 * h * h]]) / h ** 3
    m = np.array(
        [[156.0, 22.0 * h, 54.0, -13.0 * h],
         [22.0 * h, 4.0 * h * h, 13.0 * h, -3.0 * h * h],
         [54.0, 13.0 * h, 156.0, -22.0 * h],
         [-13.0 * h, -3.0 * h * h, -22.0 * h, 4.0 * h * h]]) * (h / 420.0)
    return k, m


def beam_pattern(n_el: int):
    """Structural CSR pattern of the clamped beam with ``n_el`` elements.

    Free node q (0-based, original node q+1) couples to free nodes q-1, q, q+1.
    Returns (row_ptr, col_idx) as int32 arrays with sorted columns.
    """
    if n_el < 1:
        raise ValueError("need at least one element")
    n = 2 * n_el
    q = np.arange(n) // 2
    lo = np.maximum(q - 1, 0)
    hi = np.minimum(q + 1, n_el - 1)
    counts = 2 * (hi - lo + 1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    # columns of row r are the contiguous DOF range [2*lo, 2*hi + 1]
    rows = np.repeat(np.arange(n), counts)
    offs = np.arange(nnz) - row_ptr[rows]
    col_idx = 2 * lo[rows] + offs
    if nnz >= 2 ** 31:
        raise ValueError("pattern too large for int32 indices")
    return row_ptr.astype(np.int32), col_idx.astype(np.int32)


def _assemble_blocks(n_el: int, h: float, ei: np.ndarray, rho_a: float):
    """Node-block assembly: diagonal blocks Bd[q] and upper blocks Bo[q] (q, q+1)."""
    k1, m1 = element_matrices(h)
    # per-element scaled 4x4 matrices, shape (n_el, 4, 4)
    ke = ei[:, None, None] * k1[None]
    me = np.broadcast_to(rho_a * m1, (n_el, 4, 4))
    bdk = np.zeros((n_el, 2, 2))
    bdm = np.zeros((n_el, 2, 2))
    bok = np.zeros((max(n_el - 1, 0), 2, 2))
    bom = np.zeros((max(n_el - 1, 0), 2, 2))
    # element e joins original nodes e and e+1, i.e. free nodes e-1 and e.
    bdk[:] += ke[:, 2:, 2:]
    bdm[:] += me[:, 2:, 2:]
    if n_el > 1:
        bdk[:-1] += ke[1:, :2, :2]
        bdm[:-1] += me[1:, :2, :2]
        bok[:] = ke[1:, :2, 2:]
        bom[:] = me[1:, :2, 2:]
    return (bdk, bok), (bdm, bom)


def _blocks_to_values(n_el: int, bd: np.ndarray, bo: np.ndarray, row_ptr, col_idx):
    """Scatter node blocks onto the structural CSR pattern (explicit zeros kept)."""
    n = 2 * n_el
    nnz = col_idx.shape[0]
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    cols = col_idx.astype(np.int64)
    qr, ir = rows // 2, rows % 2
    qc, ic = cols // 2, cols % 2
    val = np.empty(nnz)
    same = qc == qr
    val[same] = bd[qr[same], ir[same], ic[same]]
    up = qc == qr + 1
    val[up] = bo[qr[up], ir[up], ic[up]]
    dn = qc == qr - 1
    # block (q, q-1) is the transpose of the upper block (q-1, q)
    val[dn] = bo[qc[dn], ic[dn], ir[dn]]
    return val


def make_beam(n_el: int, ei=1.0, *, ei_loguniform=None, seed: int = 0,
              surrogate: bool = False, length: float = 1.0, rho_a: float = 1.0,
              alpha: float = ALPHA, beta: float = BETA, rng=None) -> Pencil:
    """Build the clamped cantilever pencil (M, K).

    ei: uniform bending stiffness (used when ``ei_loguniform`` is None).
    ei_loguniform: (lo, hi) -> per-element EI = exp(U(ln lo, ln hi)) drawn
        first from ``numpy.random.default_rng(seed)`` (or ``rng``).
    surrogate: scale every EI_e by h^4 (the well-conditioned surrogate whose
        dimensionless stiffness-to-mass ratio is O(1)).
    """
    if rng is None:
        rng = np.random.default_rng(seed)
    h = length / n_el
    if ei_loguniform is not None:
        lo, hi = ei_loguniform
        eis = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_el))
    else:
        eis = np.full(n_el, float(ei))
    if surrogate:
        eis = eis * h ** 4
    row_ptr, col_idx = beam_pattern(n_el)
    (bdk, bok), (bdm, bom) = _assemble_blocks(n_el, h, eis, rho_a)
    k_val = _blocks_to_values(n_el, bdk, bok, row_ptr, col_idx)
    m_val = _blocks_to_values(n_el, bdm, bom, row_ptr, col_idx)
    return Pencil(n=2 * n_el, row_ptr=row_ptr, col_idx=col_idx, m_val=m_val,
                  k_val=k_val, alpha=alpha, beta=beta, ei=eis)


def tip_load(n: int) -> np.ndarray:
    """SISO input: unit load on the tip deflection DOF, shape (1, n)."""
    f = np.zeros((1, n))
    f[0, n - 2] = 1.0
    return f


def node_loads(n: int, m: int, rng) -> tuple[np.ndarray, np.ndarray]:
    """MIMO input: unit deflection loads at ``m`` distinct seeded nodes.

    Nodes are drawn as rng.choice(n_el, m, replace=False) + 1 (original node
    numbering; node 0 is clamped). Returns (F of shape (m, n), nodes).
    """
    n_el = n // 2
    nodes = rng.choice(n_el, m, replace=False) + 1
    f = np.zeros((m, n))
    for c, node in enumerate(nodes):
        f[c, 2 * (int(node) - 1)] = 1.0
    return f, nodes


def log_shifts(lo_exp: float, hi_exp: float, count: int) -> np.ndarray:
    """Real expansion points log-spaced in [10^lo_exp, 10^hi_exp]."""
    return np.logspace(lo_exp, hi_exp, count)


def drift_shifts(shifts: np.ndarray, eps: float, rng) -> np.ndarray:
    """Vertical (next outer iteration) expansion points: s * (1 + eps * xi),
    xi ~ U(-1, 1), standing in for the shifts a later outer iteration would pick."""
    xi = rng.uniform(-1.0, 1.0, size=len(shifts))
    return shifts * (1.0 + eps * xi)


def pencil_dense(p: Pencil):
    """Dense (M, K) for tiny test cases."""
    n = p.n
    m = np.zeros((n, n))
    k = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(p.row_ptr))
    m[rows, p.col_idx] = p.m_val
    k[rows, p.col_idx] = p.k_val
    return m, k


# ---------------------------------------------------------------------------
# Named workloads. Each returns (pencil, F, shifts) built from one seed in a
# fixed draw order: element EI values first, then load nodes, then drifts.
# ---------------------------------------------------------------------------

WORKLOADS = {
    # name: (n_el, ei spec, m, shift spec)
    "c1": dict(n_el=500, ei=1.0, lu=None, m=1, shifts=("list", [100.0])),
    "c2": dict(n_el=50_000, ei=None, lu=(0.5, 2.0), m=1, shifts=("log", 0, 4, 8)),
    "c3": dict(n_el=500_000, ei=1.0, lu=None, m=4, shifts=("log", 0, 4, 16)),
    "c5": dict(n_el=5_000_000, ei=None, lu=(0.1, 10.0), m=4, shifts=("log", 0, 5, 32)),
}


def make_workload(name: str, *, surrogate: bool = False, seed: int = 0,
                  n_el: int | None = None):
    """Build a named workload; ``n_el`` overrides the size (same recipe)."""
    spec = WORKLOADS[name]
    rng = np.random.default_rng(seed)
    ne = spec["n_el"] if n_el is None else n_el
    pen = make_beam(ne, ei=spec["ei"] if spec["ei"] is not None else 1.0,
                    ei_loguniform=spec["lu"], surrogate=surrogate, rng=rng)
    if spec["m"] == 1:
        f = tip_load(pen.n)
    else:
        f, _ = node_loads(pen.n, spec["m"], rng)
    sh = spec["shifts"]
    shifts = np.array(sh[1], dtype=float) if sh[0] == "list" else log_shifts(*sh[1:])
    return pen, f, shifts, rng
