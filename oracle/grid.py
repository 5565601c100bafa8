"""Dense and coarse grid geometry (paper Sec. 3.1, "Grid design").

The dense grid is made first; every M-th dense face along an axis is a face of
the coarse grid, and the dense cells inside one coarse cell need not be equal.
Scalars live at dense cell centres (cell averages); velocities are face
averages on the staggered faces (Sec. 2.2, Fig. 1).  Test infrastructure only.
"""
import numpy as np


class Axis:
    """One axis: dense faces f[0..n], refinement factor m, periodic or walled.

    Attributes
      n, nc        dense and coarse cell counts (n = m * nc)
      h, c         dense widths and centres (length n)
      cf, H        coarse faces (every m-th dense face) and coarse widths
      dc           centre-to-centre distance across each dense face: for a
                   periodic axis dc[i] (i = 0..n-1) spans cells i-1 and i, with
                   cell -1 the periodic image of cell n-1; for a walled axis
                   dc has n+1 entries and the wall faces use half a width.
    """

    def __init__(self, faces, m, periodic):
        f = np.asarray(faces, dtype=np.float64)
        if f.ndim != 1 or f.size < 2 or np.any(np.diff(f) <= 0):
            raise ValueError("faces must be strictly increasing")
        n = f.size - 1
        if m < 1 or n % m:
            raise ValueError("dense cells must be a multiple of the refinement factor")
        self.faces = f
        self.n = n
        self.m = int(m)
        self.nc = n // m
        self.periodic = bool(periodic)
        self.length = f[-1] - f[0]
        self.h = np.diff(f)
        self.c = 0.5 * (f[:-1] + f[1:])
        self.cf = f[::m].copy()
        self.H = np.diff(self.cf)
        if periodic:
            prev = np.concatenate(([self.c[-1] - self.length], self.c[:-1]))
            self.dc = self.c - prev
        else:
            self.dc = np.empty(n + 1)
            self.dc[1:-1] = np.diff(self.c)
            self.dc[0] = 0.5 * self.h[0]
            self.dc[-1] = 0.5 * self.h[-1]

    def nfaces(self):
        """Number of distinct faces normal to this axis (periodic: n; walled: n+1)."""
        return self.n if self.periodic else self.n + 1

    def ncfaces(self):
        return self.nc if self.periodic else self.nc + 1


class Grid:
    """Three axes; arrays are indexed [z][y][x] (x fastest).

    By default x and y are periodic and z is walled, the setting of the
    scalar step.  The refinement also accepts walled x and y.
    """

    def __init__(self, xf, yf, zf, m=(1, 1, 1), periodic=(True, True, False)):
        mx, my, mz = m
        if periodic[2]:
            raise ValueError("z is always bounded by walls")
        self.x = Axis(xf, mx, periodic[0])
        self.y = Axis(yf, my, periodic[1])
        self.z = Axis(zf, mz, False)

    @property
    def shape(self):
        return (self.z.n, self.y.n, self.x.n)

    def vol(self):
        """Dense cell volumes hx*hy*hz, shape (nz, ny, nx)."""
        return self.z.h[:, None, None] * self.y.h[None, :, None] * self.x.h[None, None, :]

    def area_xy(self):
        """Horizontal cell areas hx*hy, shape (ny, nx)."""
        return self.y.h[:, None] * self.x.h[None, :]
