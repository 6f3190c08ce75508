"""Oracle references computed by CPU worker processes (test infrastructure).

Some oracle references of the GPU tests take a minute of single-threaded
SciPy work: the exact overlap rows of the transfer matrix on 10^4 sampled
tets of a large mesh, or the variable-coefficient MINRES solve at 128^3.  The
pool forks its workers when the test session starts, before any test touches
the GPU, and every reference the selected GPU tests will ask for is submitted
at once, so the CPU work runs while the GPU tests run.  A test then blocks on
the result it needs.  If the pool was not started (a CPU-only session, or a
run that imports this module later), a reference is computed in the calling
process instead.

Only oracle/ and the seeded input generators in workloads/ are called here.
"""
from __future__ import annotations

import math
import multiprocessing as mp
import multiprocessing.pool  # noqa: F401  (mp.pool.AsyncResult)
import os

import numpy as np

_POOL = None
_JOBS: dict = {}

# Sampled tet rows of a mesh: at least 10^4 (all of them when the mesh is smaller).
ROWS_PER_MESH = 10_000


def _workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    # a one-GPU machine grants 16 CPUs; leave one for the test process itself
    return max(1, min(15, n - 1))


# ---------------------------------------------------------------------------
# the references (module-level functions: they run in the workers)


_MESHES: dict = {}


def mesh_of(name: str):
    """The tet mesh of a workload or of a serving level (cached per process)."""
    from workloads import WORKLOADS, serve_mesh
    if name not in _MESHES:
        _MESHES[name] = serve_mesh(int(name[5:])) if name.startswith("serve") else WORKLOADS[name].mesh()
    return _MESHES[name]


def box_of(name: str) -> int:
    from workloads import WORKLOADS
    if name.startswith("serve"):
        return int(name[5:])
    return WORKLOADS[name].n


def sampled_rows(name: str, count: int = ROWS_PER_MESH) -> np.ndarray:
    """Sorted distinct tet rows of mesh `name` (seeded; all rows if fewer)."""
    _, tets = mesh_of(name)
    nt = tets.shape[0]
    if nt <= count:
        return np.arange(nt)
    return np.sort(np.random.default_rng(7).choice(nt, count, replace=False))


def _pi_chunk(name: str, n: int, rows: np.ndarray):
    from oracle import transfer as T
    xyz, tets = mesh_of(name)
    Pi = T.build_pi(xyz, tets, n, rows=rows)
    return Pi.indptr, Pi.indices, Pi.data


def _tet_volumes(name: str, rows: np.ndarray) -> np.ndarray:
    from oracle import transfer as T
    xyz, tets = mesh_of(name)
    return np.array([T.tet_volume(xyz[tets[r]]) for r in rows])


def _var_solve(n: int, lo: float, hi: float, seed_field: int, seed_xi: int, tol: float):
    """u of the cell-wise kappa system (kappa spanning [lo, hi], g = sqrt(8 pi kappa)),
    by the oracle's preconditioned MINRES with the constant-kappa S~ at the
    geometric-mean kappa (exact DCT inverse) to tol."""
    from oracle import discretize as D, minres as MR, variable as V
    from workloads import coefficient_field, xi_batch
    kap = coefficient_field(n, lo, hi, seed_field)
    g = np.sqrt(8.0 * np.pi * kap)
    xi = xi_batch(n, [seed_xi])[0]
    ops = D.assemble(n)
    A = V.system_matrix(ops, kap)
    F = V.rhs(ops, g, xi)
    kref = math.sqrt(float(kap.min()) * float(kap.max()))
    x, it, _ = MR.minres(lambda v: A @ v, F, MR.block_preconditioner(ops, kref), tol=tol)
    nfi = ops["M"].shape[0]
    return x[nfi:], it


# ---------------------------------------------------------------------------
# scheduling


def _split(rows: np.ndarray, parts: int):
    return [c for c in np.array_split(rows, parts) if c.size]


def _submit_pi(name: str, n: int | None = None):
    n = box_of(name) if n is None else n
    rows = sampled_rows(name)
    chunks = _split(rows, max(1, min(64, rows.size // 100)))
    if _POOL is None:
        return ("pi", name, rows, [_pi_chunk(name, n, c) for c in chunks], _tet_volumes(name, rows))
    res = [_POOL.apply_async(_pi_chunk, (name, n, c)) for c in chunks]
    vol = _POOL.apply_async(_tet_volumes, (name, rows))
    return ("pi", name, rows, res, vol)


def _submit_var(n: int, lo: float, hi: float, seed_field: int, seed_xi: int, tol: float):
    args = (n, lo, hi, seed_field, seed_xi, tol)
    if _POOL is None:
        return ("var", _var_solve(*args))
    return ("var", _POOL.apply_async(_var_solve, args))


def pi_key(name: str, n: int | None = None) -> str:
    return f"pi:{name}@{box_of(name) if n is None else n}"


def var_key(n: int, lo: float = 10.0, hi: float = 40.0, seed_field: int = 5, seed_xi: int = 0,
            tol: float = 1e-12) -> str:
    return f"var:{n}:{lo}:{hi}:{seed_field}:{seed_xi}:{tol}"


# References the GPU tests ask for; submitted when the session starts.
PREFETCH = [
    (pi_key("box16"), lambda: _submit_pi("box16")),
    (pi_key("box64"), lambda: _submit_pi("box64")),
    (pi_key("box128"), lambda: _submit_pi("box128")),
    (pi_key("box256"), lambda: _submit_pi("box256")),
    (pi_key("serve128"), lambda: _submit_pi("serve128")),
    (pi_key("serve128", 64), lambda: _submit_pi("serve128", 64)),
    (var_key(64), lambda: _submit_var(64, 10.0, 40.0, 5, 0, 1e-12)),
    (var_key(128), lambda: _submit_var(128, 10.0, 40.0, 5, 0, 1e-12)),
]


def start() -> None:
    """Fork the workers and submit every prefetched reference.  Call before
    anything in this process initialises the GPU."""
    global _POOL
    if _POOL is not None:
        return
    _POOL = mp.get_context("fork").Pool(_workers())
    for key, fn in PREFETCH:
        _JOBS[key] = fn()


def stop() -> None:
    global _POOL
    if _POOL is not None:
        _POOL.terminate()
        _POOL.join()
        _POOL = None


def _job(key: str, submit):
    if key not in _JOBS:
        _JOBS[key] = submit()
    return _JOBS[key]


def _get(x):
    return x.get() if isinstance(x, mp.pool.AsyncResult) else x


def transfer_rows(name: str, n: int | None = None):
    """(rows, Pi restricted to them as scipy CSR, tet volumes of the rows) for
    mesh `name` (a workload name or "serve<n>") and the n^3 box (default: the
    mesh's own box; a serving mesh also carries its level's coarse part)."""
    import scipy.sparse as sp
    n = box_of(name) if n is None else n
    job = _job(pi_key(name, n), lambda: _submit_pi(name, n))
    _, _, rows, parts, vol = job
    indptr = [np.zeros(1, np.int64)]
    cols, vals = [], []
    base = 0
    for p in parts:
        ip, ci, cv = _get(p)
        indptr.append(ip[1:] + base)
        base += ip[-1]
        cols.append(ci)
        vals.append(cv)
    Pi = sp.csr_matrix((np.concatenate(vals), np.concatenate(cols), np.concatenate(indptr)),
                       shape=(rows.size, n ** 3))
    return rows, Pi, _get(vol)


def variable_u(n: int, lo: float = 10.0, hi: float = 40.0, seed_field: int = 5, seed_xi: int = 0,
               tol: float = 1e-12):
    """(u, iterations) of the oracle's cell-wise kappa solve (see _var_solve)."""
    key = var_key(n, lo, hi, seed_field, seed_xi, tol)
    job = _job(key, lambda: _submit_var(n, lo, hi, seed_field, seed_xi, tol))
    return _get(job[1])


def volume_weighted_rel_l2(got: np.ndarray, ref: np.ndarray, vol: np.ndarray) -> float:
    """sqrt(sum vol (got - ref)^2) / sqrt(sum vol ref^2) over the sampled tets."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(math.sqrt(float(np.sum(vol * (got - ref) ** 2)) / float(np.sum(vol * ref ** 2))))
