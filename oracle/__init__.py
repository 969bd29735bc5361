"""Plain FP64 CPU oracle for the 4D generalized SUBSURF segmentation step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library and
its Python binding never import it, and it imports nothing from them.

The arithmetic lives in ``subsurf4d_oracle.c`` (plain loops, FP64,
``-ffp-contract=off``); this module loads it with ctypes and strings the
paper's steps together in the order of the implementation overview of
Sec. 3.5: initial condition -> local rescale -> local thresholding ->
presmoothing -> edge detector -> for each step {coefficients, SOR, rescale}.

Array conventions: numpy float64, x fastest, shapes given as (t, z, y, x);
"padded" arrays carry one ghost layer on every side (shape (N4+2, N3+2, N2+2,
N1+2)), "interior" arrays do not.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.environ.get("SUBSURF4D_ORACLE_LIB") or os.path.join(_HERE, "liboracle_subsurf4d.so")
_SRC_PATH = os.path.join(_HERE, "subsurf4d_oracle.c")

CENTRE_DTYPE = np.dtype([("x", "<f4"), ("y", "<f4"), ("z", "<f4"), ("frame", "<i4")])

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (generic x86-64, FP64, no contraction)."""
    from oracle.build import build_oracle

    return build_oracle(force=force)


def use_library(path: str) -> None:
    """Load the oracle from another build of the same source (the CPU-baseline
    timing build for the host); later calls go through it."""
    global _lib, _LIB_PATH
    _LIB_PATH = path
    _lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        L.oracle_owner_map.argtypes = [P, P, I, D, P]
        L.oracle_threshold.argtypes = [P, P, P, I, D, D, P, P]
        L.oracle_lhe_step.argtypes = [P, D, D, D, D, I, P, P]
        L.oracle_lhe_step.restype = I
        L.oracle_face_gradient.argtypes = [P, D, P, I, P]
        L.oracle_face_g.argtypes = [P, D, D, D, D, P, P, P]
        L.oracle_init_u.argtypes = [P, P, I, D, D, P]
        L.oracle_assemble.argtypes = [P, D, D, D, P, P, P, P, P]
        L.oracle_sor.argtypes = [P, I, D, D, I, I, P, P, P, P, P]
        L.oracle_sor.restype = I
        L.oracle_rescale.argtypes = [P, P, I, D, P, P]
        L.oracle_num_threads.restype = I
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(n) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(n, dtype=np.int32))


def padded_shape(n):
    n1, n2, n3, n4 = n
    return (n4 + 2, n3 + 2, n2 + 2, n1 + 2)


def interior_shape(n):
    n1, n2, n3, n4 = n
    return (n4, n3, n2, n1)


def _centres(cs) -> np.ndarray:
    if cs is None or len(cs) == 0:
        return np.zeros(1, dtype=CENTRE_DTYPE)
    return np.ascontiguousarray(np.asarray(cs, dtype=CENTRE_DTYPE))


def num_threads() -> int:
    return int(lib().oracle_num_threads())


# --------------------------------------------------------------- primitives


def owner_map(n, centres, r):
    """Owner ball of every interior cell (nearest containing centre), -1 if none."""
    cs = _centres(centres)
    nc = 0 if centres is None else len(centres)
    out = np.empty(interior_shape(n), dtype=np.int32)
    lib().oracle_owner_map(_ptr(_dims(n)), _ptr(cs), nc, float(r), _ptr(out))
    return out


def threshold(n, I0, centres, r, lam, owner):
    """Local thresholding of Sec. 3.1 (I^TH); interior arrays."""
    cs = _centres(centres)
    nc = 0 if centres is None else len(centres)
    I0 = np.ascontiguousarray(I0, dtype=np.float64)
    out = np.empty(interior_shape(n), dtype=np.float64)
    lib().oracle_threshold(_ptr(_dims(n)), _ptr(I0), _ptr(cs), nc, float(r), float(lam),
                           _ptr(np.ascontiguousarray(owner, dtype=np.int32)), _ptr(out))
    return out


def lhe_step(n, J, h, tau_s, omega=1.5, tol=1e-13, max_iter=100000):
    """One implicit zero-Neumann heat step (presmoothing, Sec. 3.1); interior arrays.

    omega <= 0 selects Young's optimal relaxation for a consistently ordered
    matrix with Jacobi spectral radius rho: 2/(1+sqrt(1-rho^2)), here with the
    interior radius rho = 8a/(1+8a), a = tau_s/h^2 (8 neighbours in 4D)."""
    if omega <= 0.0:
        a = tau_s / (h * h)
        rho = 8.0 * a / (1.0 + 8.0 * a)
        omega = 2.0 / (1.0 + np.sqrt(1.0 - rho * rho))
    J = np.ascontiguousarray(J, dtype=np.float64)
    out = np.empty_like(J)
    it = lib().oracle_lhe_step(_ptr(_dims(n)), float(h), float(tau_s), float(omega), float(tol),
                               int(max_iter), _ptr(J), _ptr(out))
    if it < 0:
        raise RuntimeError("oracle LHE solve did not converge")
    return out, it


def face_gradient(n, v_padded, d, h=1.0):
    """Reduced-diamond-cell gradient (4 components) on every '+e_d' face."""
    v = np.ascontiguousarray(v_padded, dtype=np.float64)
    out = np.empty(padded_shape(n) + (4,), dtype=np.float64)
    lib().oracle_face_gradient(_ptr(_dims(n)), float(h), _ptr(v), int(d), _ptr(out))
    return out


def face_g(n, Is0, IsTH, h, K, delta, vartheta):
    """Edge detector G_d on the '+e_d' face of every padded cell; shape (4,)+padded."""
    a = np.ascontiguousarray(Is0, dtype=np.float64)
    b = np.ascontiguousarray(IsTH, dtype=np.float64)
    out = np.empty((4,) + padded_shape(n), dtype=np.float64)
    lib().oracle_face_g(_ptr(_dims(n)), float(h), float(K), float(delta), float(vartheta),
                        _ptr(a), _ptr(b), _ptr(out))
    return out


def init_u(n, seeds, v, R):
    """Initial segmentation function (peak profile around the frame's seeds)."""
    cs = _centres(seeds)
    nc = 0 if seeds is None else len(seeds)
    out = np.empty(padded_shape(n), dtype=np.float64)
    lib().oracle_init_u(_ptr(_dims(n)), _ptr(cs), nc, float(v), float(R), _ptr(out))
    return out


def assemble(n, G, w, h, eps, tau, ub=None):
    """Coefficients (interior x 8) and right-hand side of one step's system."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    ub = w if ub is None else np.ascontiguousarray(ub, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64)
    coef = np.empty(interior_shape(n) + (8,), dtype=np.float64)
    b = np.empty(interior_shape(n), dtype=np.float64)
    lib().oracle_assemble(_ptr(_dims(n)), float(h), float(eps), float(tau), _ptr(G), _ptr(w),
                          _ptr(ub), _ptr(coef), _ptr(b))
    return coef, b


LEX, RB = 0, 1


def sor(n, coef, b, u0, omega, tol, max_iter=10000, order=RB, check_every=1):
    """SOR solve (lexicographic or red-black); returns (u padded, iterations, rel_res, status)."""
    u = np.array(u0, dtype=np.float64, copy=True, order="C")
    it = ctypes.c_int(0)
    rr = ctypes.c_double(0.0)
    st = lib().oracle_sor(_ptr(_dims(n)), int(order), float(omega), float(tol), int(max_iter),
                          int(check_every), _ptr(np.ascontiguousarray(coef)),
                          _ptr(np.ascontiguousarray(b)), _ptr(u), ctypes.byref(it),
                          ctypes.byref(rr))
    return u, it.value, rr.value, st


def rescale(n, u_padded, centres, r, owner):
    """Local rescaling to [0,1] per ball (owner cells only); returns a new array."""
    cs = _centres(centres)
    nc = 0 if centres is None else len(centres)
    u = np.array(u_padded, dtype=np.float64, copy=True, order="C")
    lib().oracle_rescale(_ptr(_dims(n)), _ptr(cs), nc, float(r),
                         _ptr(np.ascontiguousarray(owner, dtype=np.int32)), _ptr(u))
    return u


# ------------------------------------------------------------------ pipeline


@dataclass(frozen=True)
class PrepareParams:
    K: float = 1000.0
    delta: float = 0.5
    vartheta: float = 0.5
    lam: float = 0.5
    ball_r: float = 8.0
    smooth_tau: float = 0.1
    smooth_steps: int = 1
    smooth_omega: float = 0.0          # <= 0: Young's optimal omega for the heat system
    smooth_tol: float = 1e-13
    h: float = 1.0


@dataclass(frozen=True)
class StepParams:
    eps: float = 1e-3
    tau: float = 0.5
    omega: float = 1.5
    tol: float = 1e-8
    max_iter: int = 10000
    check_every: int = 1
    rescale: bool = True
    ball_r: float = 8.0
    h: float = 1.0


def prepare(n, image, centres, p: PrepareParams):
    """Owner map, I^TH, presmoothed I0 and I^TH, face field G (Sec. 3.1, 3.2.2)."""
    I0 = np.ascontiguousarray(image, dtype=np.float64).reshape(interior_shape(n))
    owner = owner_map(n, centres, p.ball_r)
    ITH = threshold(n, I0, centres, p.ball_r, p.lam, owner)
    Is0, IsTH = I0, ITH
    for _ in range(p.smooth_steps):
        Is0, _ = lhe_step(n, Is0, p.h, p.smooth_tau, p.smooth_omega, p.smooth_tol)
        IsTH, _ = lhe_step(n, IsTH, p.h, p.smooth_tau, p.smooth_omega, p.smooth_tol)
    G = face_g(n, Is0, IsTH, p.h, p.K, p.delta, p.vartheta)
    return dict(owner=owner, ITH=ITH, Is0=Is0, IsTH=IsTH, G=G)


def step(n, G, w, centres, owner, p: StepParams, order=RB, fixed_iters=None):
    """One semi-implicit step: assemble, SOR, local rescale.

    ``fixed_iters`` runs exactly that many iterations (tol=0) instead of the
    stopping rule.  Returns a dict with u (before rescale), u_resc, iterations,
    rel_res, status.
    """
    coef, b = assemble(n, G, w, p.h, p.eps, p.tau)
    if fixed_iters is None:
        u, it, rr, st = sor(n, coef, b, w, p.omega, p.tol, p.max_iter, order, p.check_every)
    else:
        u, it, rr, st = sor(n, coef, b, w, p.omega, 0.0, int(fixed_iters), order, 1)
        st = 0
    ur = rescale(n, u, centres, p.ball_r, owner) if p.rescale else u.copy()
    return dict(u=u, u_resc=ur, iterations=it, rel_res=rr, status=st)


def run(n, image, centres, seeds, pp: PrepareParams, sp: StepParams, steps, v=1.0, R=0.0,
        order=RB, record=True):
    """Driver of Sec. 3.5: u0 -> rescale -> ``steps`` x (assemble, SOR, rescale)."""
    prep = prepare(n, image, centres, pp)
    u0 = init_u(n, seeds, v, R)
    w = rescale(n, u0, centres, sp.ball_r, prep["owner"]) if sp.rescale else u0
    out = dict(prep=prep, u0=u0, w0=w, steps=[])
    for _ in range(steps):
        rec = step(n, prep["G"], w, centres, prep["owner"], sp, order)
        w = rec["u_resc"]
        out["steps"].append(rec if record else dict(iterations=rec["iterations"],
                                                    rel_res=rec["rel_res"]))
    out["u_final"] = w
    return out


# ----------------------------------------------------------- dense reference


def dense_system(n, coef, b):
    """Interior matrix A and rhs b of the step system as dense numpy arrays.

    Row P: A[P,P] = 1 + sum of its 8 coefficients, A[P,nbr] = -c for interior
    neighbours (ghost terms are already in b).  For tiny grids only.
    """
    n1, n2, n3, n4 = n
    N = n1 * n2 * n3 * n4
    A = np.zeros((N, N))
    cf = np.asarray(coef).reshape(N, 8)
    strides = (1, n1, n1 * n2, n1 * n2 * n3)
    for q in range(N):
        idx = [q % n1, (q // n1) % n2, (q // (n1 * n2)) % n3, q // (n1 * n2 * n3)]
        A[q, q] = 1.0 + cf[q].sum()
        for f in range(8):
            d, s = f // 2, (1 if f & 1 else -1)
            t = idx[d] + s
            if 0 <= t < n[d]:
                A[q, q + s * strides[d]] = -cf[q, f]
    return A, np.asarray(b).reshape(N).copy()


def interior(a_padded):
    return np.ascontiguousarray(a_padded[1:-1, 1:-1, 1:-1, 1:-1])


# ---------------------------------------------------------------- EOC test


def eoc_run(N, steps, T=0.0625, L=1.25, omega=1.5, tol=1e-11, grid="cell", eps=None, lagged_dirichlet=False):
    """Sec. 3.4: level-set mean-curvature flow with the exact solution
    u = (x1^2+x2^2+x3^2+x4^2 - 1)/6 + t on [-L, L]^4, G = 1, tau = T/steps,
    Dirichlet data from the exact solution, no rescaling.  Returns the
    L2(0,T;L2) error sqrt(sum_n tau * sum_P h^4 (u^n_P - u(x_P, t_n))^2) and
    the SOR iteration counts.

    The paper states the domain, N, the step counts, eps = h^2 and the norm,
    not where the unknowns sit or when the boundary data are taken.  Readings:
    grid="cell" (default): N cells of width h = 2L/N, centres
    x_i = -L + (i - 1/2) h, ghost centres one h outside; grid="node": nodes
    x_i = -L + i h, i = 0..N, with the N-1 interior nodes unknown and the
    nodes on the boundary holding the data.  The ghosts of u^{n-1} (they feed
    the boundary-face gradients) hold the exact solution at t_{n-1}; the
    Dirichlet data of the new level are the exact solution at t_n, or at
    t_{n-1} with lagged_dirichlet=True.  eps defaults to h^2.
    """
    h = 2 * L / N
    if grid == "cell":
        x = -L + (np.arange(N + 2) - 0.5) * h
        n = (N, N, N, N)
    elif grid == "node":
        x = -L + np.arange(N + 1) * h
        n = (N - 1,) * 4
    else:
        raise ValueError(grid)
    eps = h * h if eps is None else float(eps)
    X4, X3, X2, X1 = np.meshgrid(x, x, x, x, indexing="ij")
    r2 = X1 ** 2 + X2 ** 2 + X3 ** 2 + X4 ** 2
    exact = lambda t: (r2 - 1.0) / 6.0 + t  # noqa: E731
    tau = T / steps
    G = np.ones((4,) + padded_shape(n))
    w = exact(0.0)
    inner = (slice(1, -1),) * 4
    err2 = 0.0
    its = []
    for s in range(1, steps + 1):
        ub = exact((s - 1) * tau if lagged_dirichlet else s * tau)
        coef, b = assemble(n, G, w, h, eps, tau, ub=ub)
        u0 = ub.copy()
        u0[inner] = w[inner]
        u, it, rr, st = sor(n, coef, b, u0, omega, tol, 100000, RB)
        its.append(it)
        ex = exact(s * tau)
        e = interior(u) - interior(ex)
        err2 += tau * (h ** 4) * float(np.sum(e * e))
        w = ex.copy()                      # next level's gradient ghosts: exact solution at t_s
        w[inner] = u[inner]
    return float(np.sqrt(err2)), its


# ------------------------------------------------------------ cell tracking

CELL_DTYPE = np.dtype([("name", "<i4"), ("frame", "<i4"), ("centre", "<i4"), ("d2", "<i4"), ("prev", "<i4"),
                       ("kind", "<i4")])


def track_label(n, u_padded, level):
    """Cells of every frame (Sec. 5): 6-connected sets of voxels with u >= level,
    each voxel labelled with its cell's smallest interior index, -1 outside."""
    L = lib()
    L.oracle_track_label.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p]
    u = np.ascontiguousarray(u_padded, dtype=np.float64)
    out = np.empty(interior_shape(n), dtype=np.int32)
    L.oracle_track_label(_ptr(_dims(n)), _ptr(u), float(level), _ptr(out))
    return out


def track_dist2(n, label):
    """Squared distance of every cell voxel to the nearest voxel outside its cell."""
    L = lib()
    L.oracle_track_dist2.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lab = np.ascontiguousarray(label, dtype=np.int32)
    out = np.empty(interior_shape(n), dtype=np.int32)
    L.oracle_track_dist2(_ptr(_dims(n)), _ptr(lab), _ptr(out))
    return out


def track_cells(n, label, d2, capacity=1 << 16):
    """Per-cell records (name, frame, centre, d2, prev, kind) in name order."""
    L = lib()
    L.oracle_track_cells.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_int]
    L.oracle_track_cells.restype = ctypes.c_int
    rec = np.zeros((capacity, 6), dtype=np.int32)
    k = L.oracle_track_cells(_ptr(_dims(n)), _ptr(np.ascontiguousarray(label, dtype=np.int32)),
                             _ptr(np.ascontiguousarray(d2, dtype=np.int32)), _ptr(rec), int(capacity))
    if k < 0:
        raise RuntimeError("more cells than the capacity")
    return np.ascontiguousarray(rec[:k]).view(CELL_DTYPE).reshape(k)


def voxel_xyz(n, index):
    """(x, y, z) voxel coordinates of an interior index (frame dropped)."""
    n1, n2, n3, _ = n
    q = int(index) % (n1 * n2 * n3)
    return (q % n1, (q // n1) % n2, q // (n1 * n2))


def track_join(n, cells, radius):
    """Trajectories from the backward links (Sec. 5): every cell that no cell of
    the next frame links to ends a partial trajectory, which follows the links
    back to a cell without one.  A partial trajectory T whose first cell is in
    frame f > 0 is then joined after the partial trajectory S that ends in frame
    f-1 when the tangent prolongation of one reaches the other: T's first point
    moved back by its first displacement (2 c0 - c1, or c0 for a single cell)
    lies within `radius` of S's last point, or S's last point moved on by its
    last displacement lies within `radius` of T's first point.  T takes the
    candidate with the smallest squared distance (ties: the smallest name of
    S's last cell); each S is joined at most once, T in order of the name of
    its first cell.  Returns a list of trajectories, each a list of cell
    names from the first frame to the last."""
    by_name = {int(c["name"]): c for c in cells}
    has_next = {int(c["prev"]) for c in cells if c["prev"] >= 0}
    partial = []
    for c in sorted(cells, key=lambda c: int(c["name"])):
        if int(c["name"]) in has_next:
            continue
        chain = [int(c["name"])]
        while by_name[chain[-1]]["prev"] >= 0:
            chain.append(int(by_name[chain[-1]]["prev"]))
        partial.append(chain[::-1])

    def xyz(name):
        return np.array(voxel_xyz(n, by_name[name]["centre"]), dtype=np.int64)

    ends = {}
    for t, ch in enumerate(partial):
        ends.setdefault(int(by_name[ch[-1]]["frame"]), []).append(t)
    joined_after = {}
    used = set()
    for t in sorted(range(len(partial)), key=lambda t: partial[t][0]):
        first = partial[t][0]
        f = int(by_name[first]["frame"])
        if f == 0:
            continue
        c0 = xyz(first)
        back = 2 * c0 - xyz(partial[t][1]) if len(partial[t]) > 1 else c0
        best = None
        for s in ends.get(f - 1, []):
            if s in used or s == t:
                continue
            last = partial[s][-1]
            e0 = xyz(last)
            fwd = 2 * e0 - xyz(partial[s][-2]) if len(partial[s]) > 1 else e0
            dd = min(int(np.sum((back - e0) ** 2)), int(np.sum((fwd - c0) ** 2)))
            if dd <= radius * radius and (best is None or (dd, last) < (best[0], best[1])):
                best = (dd, last, s)
        if best is not None:
            used.add(best[2])
            joined_after[t] = best[2]
    heads = [t for t in range(len(partial)) if t not in used]
    out = []
    for t in heads:
        chain = list(partial[t])
        cur = t
        while cur in joined_after:
            cur = joined_after[cur]
            chain = partial[cur] + chain
        out.append(chain)
    out.sort(key=lambda ch: ch[0])
    return out


def track(n, u_padded, level=0.5, radius=0.0):
    """The whole tracking of Sec. 5: labels, distances, cells with links, trajectories."""
    label = track_label(n, u_padded, level)
    d2 = track_dist2(n, label)
    cells = track_cells(n, label, d2)
    return dict(label=label, d2=d2, cells=cells, tracks=track_join(n, cells, radius))
