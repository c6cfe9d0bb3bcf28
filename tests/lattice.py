"""A periodic lattice whose Love-Weber stress is known in closed form.

n^3 equal spheres on a rectangular lattice in a periodic cell, spaced
a_x = 2r - delta along x (so neighbours along x overlap by delta) and
a_y = a_z = 2r + gap across (no contact).  Every x-contact gets a preset
shear force of size fs along y, oriented like a uniform shear: the force on
the right-hand sphere points along +y.  Records follow the contact-key
convention of both implementations: #1 = lower id, `cell` = the periodic
image of #2 seen from #1, normal from #1 to #2.  Geometry only.
"""
import numpy as np


def sheared_lattice(delta=2e-6, fs=1e-3, gap=0.2e-3, r=1e-3, n=5, young=1e7):
    ax, ay = 2 * r - delta, 2 * r + gap
    idx = np.array([(i, j, k) for k in range(n) for j in range(n) for i in range(n)], dtype=float)
    spacing = np.array([ax, ay, ay])
    pos = idx * spacing + 0.5 * spacing
    ident = lambda i, j, k: i + n * (j + n * k)
    id1, id2, cell, F, N = [], [], [], [], []
    for k in range(n):
        for j in range(n):
            for i in range(n):
                a, b = ident(i, j, k), ident((i + 1) % n, j, k)
                if i + 1 < n:   # #1 on the left, normal +x
                    id1.append(a), id2.append(b), cell.append((0, 0, 0)), N.append((1.0, 0, 0))
                    F.append((0, fs, 0))
                else:           # wrap pair: #1 = lower id (i = 0), #2 seen one cell to the left
                    id1.append(b), id2.append(a), cell.append((-1, 0, 0)), N.append((-1.0, 0, 0))
                    F.append((0, -fs, 0))
    return {"hsize": np.diag([n * ax, n * ay, n * ay]), "pos": pos, "radius": np.full(n ** 3, r),
            "id1": np.array(id1), "id2": np.array(id2), "cell": np.array(cell), "fs": np.array(F, dtype=float),
            "nprev": np.array(N), "ax": ax, "ay": ay, "young": young}
