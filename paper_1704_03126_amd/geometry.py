"""Seeded synthetic inputs: staircase solid masks and rarefaction fields.

This module only *generates inputs*. It holds none of the kinetic method's
arithmetic and is the one module that both the GPU solver's tests and the CPU
oracle's tests draw their inputs from.

The paper (Sec. III, Fig. 4) runs its porous-media cases on figure-only
geometries that are not available; the generators below are synthetic
stand-ins of the same kind: a periodic unit cell of side H whose solid phase is
a union of overlapping discs, rendered as a Cartesian staircase (the paper's
"stair case" wall approximation of Sec. II.A), and a channel of height H whose
walls carry rectangular roughness.

Conventions shared by every generator:
  * ``mask`` is a ``uint8`` array of shape ``(ny, nx)``, row-major, ``1`` = solid.
  * x (axis 1) is the flow direction and is always periodic.
  * ``periodic_y`` tells whether the y axis is periodic (porous cells) or
    bounded by walls on the outer faces (channels).
  * ``cells_per_H`` is the number of cells per reference length H.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Geometry:
    mask: np.ndarray            # (ny, nx) uint8, 1 = solid
    periodic_y: bool
    cells_per_H: float
    name: str = ""
    porosity: float = float("nan")
    seed: int | None = None
    meta: dict = field(default_factory=dict)

    @property
    def nx(self) -> int:
        return int(self.mask.shape[1])

    @property
    def ny(self) -> int:
        return int(self.mask.shape[0])

    @property
    def n_fluid(self) -> int:
        return int((self.mask == 0).sum())


def plane_channel(ny: int, nx: int = 1) -> Geometry:
    """Two smooth parallel walls on the outer y faces, H = ny cells."""
    m = np.zeros((ny, nx), dtype=np.uint8)
    return Geometry(m, periodic_y=False, cells_per_H=float(ny),
                    name=f"plane_channel_{nx}x{ny}", porosity=1.0)


def rough_channel(nx: int, ny: int, rough_rows: int, rough_cols: int,
                  col0: int = 0) -> Geometry:
    """Channel of height H = ny cells with aligned rectangular blocks.

    Both walls carry a block ``rough_rows`` cells high spanning columns
    ``[col0, col0 + rough_cols)``; the blocks are aligned so the geometry is
    mirror-symmetric about the channel centreline.
    """
    if not (0 <= rough_rows < ny // 2 and 0 <= rough_cols <= nx):
        raise ValueError("roughness does not fit the channel")
    m = np.zeros((ny, nx), dtype=np.uint8)
    if rough_rows > 0 and rough_cols > 0:
        cols = (np.arange(col0, col0 + rough_cols) % nx)
        m[:rough_rows, cols] = 1
        m[ny - rough_rows:, cols] = 1
    phi = float((m == 0).mean())
    return Geometry(m, periodic_y=False, cells_per_H=float(ny),
                    name=f"rough_channel_{nx}x{ny}_r{rough_rows}x{rough_cols}",
                    porosity=phi)


def wm_profile(x, A: float, D: float = 1.5, gamma: float = 1.5, n1: int = -4,
               n_max: int = 0) -> np.ndarray:
    """Weierstrass-Mandelbrot roughness r(x) of Eq. (WM), x = x1/H:
    A * sum_{n=n1}^{n_max} cos(2 pi gamma^n x) / gamma^((2-D) n)."""
    x = np.asarray(x, dtype=np.float64)
    r = np.zeros_like(x)
    for n in range(n1, n_max + 1):
        r += np.cos(2.0 * np.pi * gamma ** n * x) / gamma ** ((2.0 - D) * n)
    return A * r


def fractal_couette_channel(cells_per_H: int, aspect: int = 5, D: float = 1.5,
                            eps: float = 0.02, gamma: float = 1.5,
                            n1: int = -4) -> Geometry:
    """Channel of Sec. II: a smooth top plate at x2 = H and a bottom plate
    whose surface is the Weierstrass-Mandelbrot profile r(x1/H) of Eq. (WM),
    rendered as a staircase; length aspect * H (periodic along x).

    Readings (the paper gives the series and eps = sigma/H only):
      * the series is cut where a wavelength would drop below two cells,
        gamma^n <= cells_per_H / 2;
      * A is set so that the root mean square of r over the cell centres of
        the period equals eps * H;
      * H is measured from the mean line x2 = 0 of the bottom plate to the
        top plate; cells whose centre lies below r are solid, and rows are
        added below x2 = 0 down to the deepest valley.
    """
    nx = int(aspect * cells_per_H)
    n_max = int(np.floor(np.log(cells_per_H / 2.0) / np.log(gamma)))
    xc = (np.arange(nx) + 0.5) / cells_per_H
    unit = wm_profile(xc, 1.0, D, gamma, n1, n_max)
    A = eps / np.sqrt(np.mean(unit ** 2))
    r = A * unit                                  # in units of H
    nb = max(0, int(np.ceil(-r.min() * cells_per_H)))
    ny = nb + int(cells_per_H)
    yc = (np.arange(ny) - nb + 0.5) / cells_per_H  # centre heights, in units of H
    m = (yc[:, None] < r[None, :]).astype(np.uint8)
    return Geometry(m, periodic_y=False, cells_per_H=float(cells_per_H),
                    name=f"wm_couette_{nx}x{ny}_D{D}_eps{eps}",
                    porosity=float((m == 0).mean()),
                    meta={"A": float(A), "n_max": n_max, "rows_below": nb, "profile": r})


def graded_fractal_couette_channel(nx_per_H: int = 64, n_band: int = 60, n_rest: int = 100,
                                    aspect: int = 5, D: float = 1.5, eps: float = 0.02,
                                    gamma: float = 1.5, n1: int = -4) -> Geometry:
    """The channel of fractal_couette_channel on rows of unequal height, the
    kind of grid Sec. II.A describes: n_band rows of equal height across the
    rough band (from the deepest valley to the highest peak of r) and n_rest
    rows of equal height from there to the top plate at x2 = H; nx_per_H
    columns per H along the flow.  ``meta["dy"]`` holds the row heights in
    units of H (bottom row first) for dvm_set_row_heights."""
    nx = int(aspect * nx_per_H)
    n_max = int(np.floor(np.log(nx_per_H / 2.0) / np.log(gamma)))
    xc = (np.arange(nx) + 0.5) / nx_per_H
    unit = wm_profile(xc, 1.0, D, gamma, n1, n_max)
    A = eps / np.sqrt(np.mean(unit ** 2))
    r = A * unit
    lo, hi = float(r.min()), float(r.max())
    edges = np.concatenate([np.linspace(lo, hi, n_band + 1), np.linspace(hi, 1.0, n_rest + 1)[1:]])
    dy = np.diff(edges)
    yc = 0.5 * (edges[1:] + edges[:-1])
    m = (yc[:, None] < r[None, :]).astype(np.uint8)
    return Geometry(m, periodic_y=False, cells_per_H=float(nx_per_H),
                    name=f"wm_couette_graded_{nx}x{n_band + n_rest}_D{D}_eps{eps}",
                    porosity=float((m == 0).mean()),
                    meta={"A": float(A), "n_max": n_max, "profile": r, "dy": dy, "edges": edges})


def component_labels(mask: np.ndarray, periodic_y: bool):
    """Label 4-connected fluid components on the (x-periodic) grid.

    Returns ``(labels, percolates)`` where ``labels`` is an int32 array (-1 in
    solids) and ``percolates[i]`` is True when component ``i`` connects to its
    own translate by a non-zero multiple of the period in x, i.e. it carries a
    net flux along x.  Each visited cell remembers how many times its path
    from the component seed wrapped around each periodic axis; meeting an
    already-labelled cell with a different x-winding proves a wrapping loop.
    """
    ny, nx = mask.shape
    labels = np.full((ny, nx), -1, dtype=np.int32)
    wind_x = np.zeros((ny, nx), dtype=np.int64)
    wind_y = np.zeros((ny, nx), dtype=np.int64)
    fluid = (mask == 0)
    percolates: list[bool] = []
    for sy in range(ny):
        for sx in range(nx):
            if not fluid[sy, sx] or labels[sy, sx] >= 0:
                continue
            lab = len(percolates)
            perc = False
            labels[sy, sx] = lab
            wind_x[sy, sx] = 0
            wind_y[sy, sx] = 0
            dq = deque([(sy, sx)])
            while dq:
                y, x = dq.popleft()
                wx, wy = wind_x[y, x], wind_y[y, x]
                for dy, dx in ((0, 1), (0, -1), (1, 0), (-1, 0)):
                    yy, xx = y + dy, x + dx
                    nwx, nwy = wx, wy
                    if xx < 0:
                        xx += nx
                        nwx -= 1
                    elif xx >= nx:
                        xx -= nx
                        nwx += 1
                    if yy < 0 or yy >= ny:
                        if not periodic_y:
                            continue
                        if yy < 0:
                            yy += ny
                            nwy -= 1
                        else:
                            yy -= ny
                            nwy += 1
                    if not fluid[yy, xx]:
                        continue
                    if labels[yy, xx] < 0:
                        labels[yy, xx] = lab
                        wind_x[yy, xx] = nwx
                        wind_y[yy, xx] = nwy
                        dq.append((yy, xx))
                    elif wind_x[yy, xx] != nwx:
                        perc = True
            percolates.append(perc)
    return labels, np.array(percolates, dtype=bool)


def fill_nonpercolating(mask: np.ndarray, periodic_y: bool) -> np.ndarray:
    """Turn every fluid component that does not percolate in x into solid."""
    labels, perc = component_labels(mask, periodic_y)
    out = mask.copy()
    if perc.size:
        dead = ~perc[np.maximum(labels, 0)] & (labels >= 0)
        out[dead] = 1
    return out


def porous_discs(n: int, porosity: float, seed: int,
                 rmin: float = 0.03, rmax: float = 0.08,
                 max_redraw: int = 64) -> Geometry:
    """Periodic n x n unit cell of overlapping random discs.

    Disc centres are uniform in the unit square and radii uniform in
    ``[rmin, rmax]`` times the side, drawn from ``numpy.random.default_rng``
    (PCG64).  A cell is solid when its centre lies within the periodic
    distance r of a disc centre.  Discs are added until the fluid fraction
    first drops to ``porosity`` or below; fluid components that do not
    percolate in x are then filled.  If no component percolates the draw is
    repeated with ``seed + 1``.  The final porosity is reported.
    """
    c = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(c, c)  # (ny, nx): X varies along axis 1
    for attempt in range(max_redraw):
        s = seed + attempt
        rng = np.random.default_rng(s)
        solid = np.zeros((n, n), dtype=bool)
        while (~solid).mean() > porosity:
            cx, cy = rng.random(2)
            r = rng.uniform(rmin, rmax)
            dx = np.abs(X - cx)
            dx = np.minimum(dx, 1.0 - dx)
            dy = np.abs(Y - cy)
            dy = np.minimum(dy, 1.0 - dy)
            solid |= (dx * dx + dy * dy) <= r * r
        m = solid.astype(np.uint8)
        m = fill_nonpercolating(m, periodic_y=True)
        if (m == 0).any():
            phi = float((m == 0).mean())
            return Geometry(m, periodic_y=True, cells_per_H=float(n),
                            name=f"porous_{n}_phi{porosity}_seed{seed}",
                            porosity=phi, seed=s)
    raise RuntimeError("no percolating porous cell found")


def delta_field(shape, seed: int, mean: float = 1.0, amp: float = 0.2,
                sigma: float = 8.0) -> np.ndarray:
    """Log-normal rarefaction field delta(x) = mean * exp(amp * g).

    g is iid N(0,1) per cell, smoothed by a periodic Gaussian filter of
    standard deviation ``sigma`` cells, then re-standardised to zero mean and
    unit standard deviation.
    """
    ny, nx = shape
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((ny, nx))
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.fftfreq(nx)[None, :]
    filt = np.exp(-2.0 * (np.pi * sigma) ** 2 * (kx * kx + ky * ky))
    gs = np.fft.ifft2(np.fft.fft2(g) * filt).real
    gs = (gs - gs.mean()) / gs.std()
    return mean * np.exp(amp * gs)


def cfg_plane_channel() -> Geometry:
    """1 periodic cell x 64 cells across H (x-invariant plane channel)."""
    return plane_channel(64, 1)


def cfg_rough_channel(nx: int = 256, ny: int = 128) -> Geometry:
    """2H x H periodic cell with blocks 0.2H high over half the period."""
    return rough_channel(nx, ny, int(round(0.2 * ny)), nx // 2)


def cfg_porous(n: int = 512, porosity: float = 0.6, seed: int = 1003) -> Geometry:
    return porous_discs(n, porosity, seed)


def batch_instances(count: int = 64, seed: int = 1004, smin: int = 64,
                    smax: int = 384) -> list:
    """Uneven batch: alternating porous cells and rough channels.

    Instance i uses geometry seed ``seed + i``.  Side s is uniform on the
    integers [smin, smax]; even i is an s x s porous cell (porosity 0.6), odd
    i an s x s/2 rough channel whose blocks are round(0.2 ny) rows by s/2
    columns.  delta is log-uniform on [0.01, 100].
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        s = int(rng.integers(smin, smax + 1))
        dlt = float(10.0 ** rng.uniform(-2.0, 2.0))
        if i % 2 == 0:
            g = porous_discs(s, 0.6, seed + i)
        else:
            ny = max(s // 2, 8)
            g = rough_channel(s, ny, int(round(0.2 * ny)), s // 2)
        g.meta["delta"] = dlt
        out.append(g)
    return out
