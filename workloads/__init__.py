"""Seeded synthetic inputs for the BDDC-SO model problem.

This module is shared by the CPU oracle and by the GPU path.  It only draws
random numbers and lays out descriptor arrays (mesh sizes, element->subdomain
and element->subsubdomain ids, per-element coefficients, nodal right-hand
sides).  It holds none of the method's arithmetic: no element matrices, no
classification of interface nodes, no weights, no solves.

Conventions (both consumers rely on them):

* Structured mesh on the unit square / cube with ``n_el = (nx, ny[, nz])``
  elements and spacing ``h = 1/n`` per axis.  Elements are numbered
  lexicographically, x fastest: ``e = ex + nx*(ey + ny*ez)``.
* Free nodes are the grid nodes off the boundary (zero Dirichlet data on the
  whole boundary, as in the paper's model problem, Section 2); they are
  numbered lexicographically, x fastest, over ``1..n-1`` per axis.
* ``elem_sub`` (int32) gives each element its subdomain (the partition Theta,
  Section 3); ``elem_subsub`` (int32) gives its subsubdomain (the finer
  partition used to define subobjects, Section 3).  Every subsubdomain lies in
  one subdomain.
* ``rho`` (float64, one value per element) is the diffusion coefficient of
  Remark 4; ``f`` (float64, ``[nrhs, n_free]``) is the nodal load vector.

Random streams: ``numpy.random.default_rng(SeedSequence([cfg, stream]))`` with
stream 0 = f, 1 = rho, 2 = cut planes, 3 = subobject lengths, 4 = channels,
5 = theta, 6 = theta_obs, 7 = finite-difference directions.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Problem", "rng", "tensor_problem", "uniform_cuts", "refine_cuts",
    "config1", "config2", "config3", "config4", "config5",
    "config2_like", "config5_like", "fig1_problem", "table1_problem",
    "n_free_of",
]


@dataclasses.dataclass
class Problem:
    """Raw descriptors of one model problem (the inputs of the solver)."""
    dim: int
    n_el: Tuple[int, ...]          # elements per axis
    h: Tuple[float, ...]           # mesh spacing per axis
    elem_sub: np.ndarray           # int32 [n_elements]
    elem_subsub: np.ndarray        # int32 [n_elements]
    rho: np.ndarray                # float64 [n_elements]
    f: np.ndarray                  # float64 [nrhs, n_free]
    name: str = ""
    primal_mask: int = 7           # 1 = vertices, 2 = edges, 4 = faces
    weighting: int = 1             # 0 = counting (eq. W), 1 = coefficient (Remark 4)
    extra: dict = dataclasses.field(default_factory=dict)

    @property
    def n_elements(self) -> int:
        return int(np.prod(self.n_el))

    @property
    def n_free(self) -> int:
        return n_free_of(self.n_el)

    @property
    def n_sub(self) -> int:
        return int(self.elem_sub.max()) + 1


def n_free_of(n_el: Sequence[int]) -> int:
    return int(np.prod([n - 1 for n in n_el]))


def rng(cfg: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([cfg, stream]))


def uniform_cuts(n: int, size: int) -> List[int]:
    """Cut points 0, size, 2*size, ..., n of a uniform 1D partition."""
    if n % size:
        raise ValueError(f"{n} elements are not divisible into pieces of {size}")
    return list(range(0, n + 1, size))


def refine_cuts(cuts: Sequence[int], piece: int) -> List[int]:
    """Split every interval of ``cuts`` into pieces of about ``piece`` elements.

    An interval of length ``m`` gets ``p = max(1, round(m / piece))`` pieces
    with cut points ``round(j*m/p)``.
    """
    out = [int(cuts[0])]
    for a, b in zip(cuts[:-1], cuts[1:]):
        m = b - a
        p = max(1, int(round(m / piece)))
        for j in range(1, p + 1):
            out.append(int(a) + int(round(j * m / p)))
    return out


def _interval_index(n: int, cuts: Sequence[int]) -> np.ndarray:
    idx = np.empty(n, dtype=np.int64)
    for k, (a, b) in enumerate(zip(cuts[:-1], cuts[1:])):
        idx[a:b] = k
    return idx


def _tensor_ids(n_el: Sequence[int], cuts: Sequence[Sequence[int]]) -> np.ndarray:
    """Element -> cell id of the tensor partition given by per-axis cuts."""
    dim = len(n_el)
    per_axis = [_interval_index(n_el[a], cuts[a]) for a in range(dim)]
    counts = [len(cuts[a]) - 1 for a in range(dim)]
    grids = np.meshgrid(*per_axis, indexing="ij")  # axis order x, y, z
    ids = np.zeros_like(grids[0])
    stride = 1
    for a in range(dim):
        ids = ids + grids[a] * stride
        stride *= counts[a]
    # meshgrid with 'ij' gives shape (nx, ny, nz); flatten x fastest
    return np.ascontiguousarray(ids.transpose(*reversed(range(dim)))).reshape(-1).astype(np.int32)


def tensor_problem(n_el: Sequence[int], sub_cuts: Sequence[Sequence[int]],
                   fine_cuts: Sequence[Sequence[int]], *, rho=None, cfg: int = 0,
                   nrhs: int = 1, name: str = "", primal_mask: int = 7,
                   weighting: int = 1) -> Problem:
    """Problem on a tensor-product partition.

    ``sub_cuts[a]`` are the subdomain cut points along axis ``a``;
    ``fine_cuts[a]`` must contain them (the fine partition refines the
    coarse one).  ``rho`` defaults to 1.  ``f`` is i.i.d. uniform[-1, 1]
    from stream 0 of ``cfg``.
    """
    dim = len(n_el)
    for a in range(dim):
        if not set(sub_cuts[a]) <= set(fine_cuts[a]):
            raise ValueError("fine cuts must refine the subdomain cuts")
    elem_sub = _tensor_ids(n_el, sub_cuts)
    elem_subsub = _tensor_ids(n_el, fine_cuts)
    n_elem = int(np.prod(n_el))
    if rho is None:
        rho = np.ones(n_elem)
    rho = np.asarray(rho, dtype=np.float64).reshape(-1)
    f = rng(cfg, 0).uniform(-1.0, 1.0, size=(nrhs, n_free_of(n_el)))
    return Problem(dim, tuple(int(n) for n in n_el), tuple(1.0 / n for n in n_el),
                   elem_sub, elem_subsub, rho, f, name=name,
                   primal_mask=primal_mask, weighting=weighting,
                   extra={"sub_cuts": [list(c) for c in sub_cuts],
                          "fine_cuts": [list(c) for c in fine_cuts]})


def _per_sub_rho(elem_sub: np.ndarray, n_sub: int, cfg: int, lo=-3.0, hi=3.0) -> np.ndarray:
    exps = rng(cfg, 1).uniform(lo, hi, size=n_sub)
    return (10.0 ** exps)[elem_sub]


def config1() -> Problem:
    """2D 64x64, 4x4 subdomains of 16x16, subobjects of length 4h, rho = 1."""
    n = 64
    sc = uniform_cuts(n, 16)
    fc = uniform_cuts(n, 4)
    return tensor_problem((n, n), [sc, sc], [fc, fc], cfg=1, name="cfg1")


def config2_like(n: int = 96, H: int = 12, L: int = 4, cfg: int = 2, name: str = "cfg2",
                 log_range=(-3.0, 3.0)) -> Problem:
    """3D n^3, subdomains of H^3 elements, subobjects of L, rho = 10^U per subdomain."""
    sc = uniform_cuts(n, H)
    fc = uniform_cuts(n, L)
    p = tensor_problem((n, n, n), [sc] * 3, [fc] * 3, cfg=cfg, name=name)
    if log_range is not None:
        p.rho = _per_sub_rho(p.elem_sub, p.n_sub, cfg, *log_range)
    return p


def config2() -> Problem:
    """3D 96^3, 8x8x8 subdomains of 12^3, L = 4h, log10 rho ~ U[-3,3] per subdomain."""
    return config2_like(96, 12, 4, cfg=2, name="cfg2")


def config4() -> Problem:
    """Mesh, partition and rho of config 2 with subobjects of length 2h."""
    p = config2_like(96, 12, 2, cfg=2, name="cfg4")
    return p


def _draw_intervals(r: np.random.Generator, n: int, count: int, lo: int, hi: int) -> List[int]:
    while True:
        lens = r.integers(lo, hi + 1, size=count)
        if int(lens.sum()) == n:
            return [0] + [int(v) for v in np.cumsum(lens)]


def config3(n: int = 128, nrhs: int = 32, count: int = 10, cfg: int = 3,
            n_channels_per_axis: int = 4, contrast: float = 1e6) -> Problem:
    """Uneven tensor partition, per-interval subobject length, aligned channels.

    Per axis: ``count`` intervals of 8..16 elements summing to ``n`` (stream 2,
    redrawn until the sum matches).  Per (axis, interval): a subobject length
    drawn from {2, 4, 8} (stream 3).  Channels (stream 4): straight lines of
    fine cells spanning the domain, ``n_channels_per_axis`` per direction,
    with rho = ``contrast`` inside and 1 elsewhere.
    """
    r_cut = rng(cfg, 2)
    r_len = rng(cfg, 3)
    sub_cuts, fine_cuts = [], []
    for a in range(3):
        sc = _draw_intervals(r_cut, n, count, 8, 16)
        fc = [0]
        for a0, b0 in zip(sc[:-1], sc[1:]):
            L = int(r_len.choice([2, 4, 8]))
            fc.extend(refine_cuts([a0, b0], L)[1:])
        sub_cuts.append(sc)
        fine_cuts.append(fc)
    p = tensor_problem((n, n, n), sub_cuts, fine_cuts, cfg=cfg, nrhs=nrhs, name="cfg3")
    rho = np.ones((n, n, n))  # indexed [z, y, x]
    r_ch = rng(cfg, 4)
    chans = []
    for axis in range(3):
        others = [b for b in range(3) if b != axis]
        for _ in range(n_channels_per_axis):
            cell = []
            for b in others:
                k = int(r_ch.integers(0, len(fine_cuts[b]) - 1))
                cell.append((fine_cuts[b][k], fine_cuts[b][k + 1]))
            sl = [slice(None)] * 3
            for b, (lo, hi) in zip(others, cell):
                sl[2 - b] = slice(lo, hi)
            rho[tuple(sl)] = contrast
            chans.append((axis, cell))
    p.rho = rho.reshape(-1).astype(np.float64)
    p.extra["channels"] = chans
    return p


def config5_like(n: int = 64, H: int = 8, L: int = 4, cfg: int = 5, name: str = "cfg5"):
    """3D n^3, subdomains of H^3, L; raw log-coefficients theta, theta_obs ~ N(0,1).

    Returns the problem (rho left at 1: the caller maps theta to rho) and the
    two raw per-element fields.
    """
    sc = uniform_cuts(n, H)
    fc = uniform_cuts(n, L)
    p = tensor_problem((n, n, n), [sc] * 3, [fc] * 3, cfg=cfg, name=name)
    theta = rng(cfg, 5).standard_normal(p.n_elements)
    theta_obs = rng(cfg, 6).standard_normal(p.n_elements)
    p.extra["theta"] = theta
    p.extra["theta_obs"] = theta_obs
    return p


def config5() -> Problem:
    """Adjoint workload: 64^3, 8x8x8 subdomains of 8^3, L = 4h."""
    return config5_like(64, 8, 4, cfg=5, name="cfg5")


def fd_directions(cfg: int, count: int, size: int) -> np.ndarray:
    return rng(cfg, 7).standard_normal((count, size))


def fig1_problem() -> Problem:
    """The 2D example of Figure 1: a 20x20 mesh, 2x2 subdomains split at 10.

    Fine partition: the left half is cut by the polyline
    (10,5)-(5,5)-(5,10)-(5,16)-(10,16) and the right half by x = 15, giving
    eight subsubdomains numbered as in the figure.
    """
    n = 20
    ex, ey = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")  # [ey, ex]
    cx, cy = ex + 0.5, ey + 0.5
    sub = np.where(cx < 10, np.where(cy < 10, 0, 1), np.where(cy < 10, 2, 3))
    ss = np.empty_like(sub)
    left_lo = (cx < 10) & (cy < 10)
    left_hi = (cx < 10) & (cy >= 10)
    ss[left_lo] = 0
    ss[left_lo & (cx > 5) & (cy > 5)] = 1
    ss[left_hi] = 2
    ss[left_hi & (cx > 5) & (cy < 16)] = 3
    right_lo = (cx > 10) & (cy < 10)
    right_hi = (cx > 10) & (cy >= 10)
    ss[right_lo] = np.where(cx[right_lo] < 15, 4, 5)
    ss[right_hi] = np.where(cx[right_hi] < 15, 6, 7)
    f = rng(0, 0).uniform(-1, 1, size=(1, n_free_of((n, n))))
    return Problem(2, (n, n), (1.0 / n, 1.0 / n), sub.reshape(-1).astype(np.int32),
                   ss.reshape(-1).astype(np.int32), np.ones(n * n), f, name="fig1",
                   weighting=0)


def table1_problem(k: int, L: int = 4, subs_per_axis: int = 10, f_one: bool = True) -> Problem:
    """Section 5.1 setup: (10k)^3 hexahedra, 10^3 subdomains of k^3, L/h given."""
    n = subs_per_axis * k
    sc = uniform_cuts(n, k)
    fc = uniform_cuts(n, L) if k % L == 0 else refine_cuts(sc, L)
    p = tensor_problem((n, n, n), [sc] * 3, [fc] * 3, cfg=10 + k, name=f"table1_k{k}")
    if f_one:
        p.f = np.ones_like(p.f)
    return p


def config1_like(n: int = 64, H: int = 16, L: int = 4, cfg: int = 1, rho=None,
                 name: str = "cfg1", nrhs: int = 1) -> Problem:
    sc = uniform_cuts(n, H)
    fc = uniform_cuts(n, L)
    return tensor_problem((n, n), [sc, sc], [fc, fc], cfg=cfg, rho=rho, name=name, nrhs=nrhs)


def channels_problem(n: int = 40, subs: int = 4, ell: float = 6.0, width: int = 3, per_axis: int = 2,
                     cfg: int = 20, physics: bool = True, f_one: bool = True) -> Problem:
    """Section 5.2's channels problem: an n^3 mesh in subs^3 box subdomains,
    with straight channels of coefficient 10^ell in a background of 1.  Per
    axis direction, ``per_axis`` channels of ``width`` x ``width`` elements
    run through the whole domain at positions drawn from stream 4 of ``cfg``
    (the paper's figure of the geometry is not in the text), centred in
    a row of subdomains drawn from stream 4 of ``cfg``, so that no channel
    runs along an interface plane.

    ``physics=True``: every subdomain is split into its background part and
    its channel part (which may be several disconnected pieces), and these
    are the subsubdomains (BDDC-SO with physics-based subobjects).
    ``physics=False``: the subsubdomains are the subdomains (standard BDDC).
    f = 1 at every free node (the paper's load) unless ``f_one`` is False."""
    n_el = (n, n, n)
    cuts = uniform_cuts(n, n // subs)
    elem_sub = _tensor_ids(n_el, [cuts] * 3)
    e = np.arange(n ** 3)
    ec = np.stack([e % n, (e // n) % n, e // (n * n)], axis=1)
    r = rng(cfg, 4)
    chan = np.zeros(n ** 3, dtype=bool)
    lines = []
    H = n // subs
    off = (H - width) // 2
    for a in range(3):
        b, c = [x for x in range(3) if x != a]
        for _ in range(per_axis):
            p, q = (int(v) * H + off for v in r.integers(0, subs, size=2))
            lines.append((a, p, q))
            chan |= (ec[:, b] >= p) & (ec[:, b] < p + width) & (ec[:, c] >= q) & (ec[:, c] < q + width)
    rho = np.where(chan, 10.0 ** ell, 1.0)
    if physics:
        raw = 2 * elem_sub.astype(np.int64) + chan.astype(np.int64)
        _, elem_subsub = np.unique(raw, return_inverse=True)
        elem_subsub = elem_subsub.reshape(-1).astype(np.int32)
    else:
        elem_subsub = elem_sub.copy()
    nf = n_free_of(n_el)
    f = np.ones((1, nf)) if f_one else rng(cfg, 0).uniform(-1.0, 1.0, size=(1, nf))
    return Problem(3, n_el, (1.0 / n,) * 3, elem_sub, elem_subsub, rho, f,
                   name=f"channels_n{n}_l{ell:g}_{'so' if physics else 'std'}",
                   primal_mask=4 if physics else 7, weighting=1,
                   extra={"channels": lines, "width": width})
