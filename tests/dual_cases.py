"""Hand-built field states for the dual-mesh tests (no method arithmetic:
each vertex takes its geodesically nearest seed's layer, plus a band of the
next ones, on a unit sphere)."""
import numpy as np

from paper_1804_09152_amd import inputs as I

# +x, -x, +y, -y, +z, -z, then the centre of the octant (+x, +y, +z)
OCTA_DIRS = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                      [1, 1, 1]], float)


def octahedron_plus_face(level=4, delta=0.08):
    """Seven cells on a unit icosphere: the six octahedron directions and one
    small cell at the centre of the octant (+x, +y, +z).  Each vertex holds
    its nearest seed (weight 1) and every seed whose angular distance is
    within `delta` of the nearest (weight 0.6), normalised: two-way bands
    (0.625 / 0.375) and three-way junctions (0.45 / 0.27 / 0.27), all above
    the dual-mesh threshold 0.25.

    The seventh cell touches exactly the three octahedron cells around it,
    which touch each other: the 3-clique of those three covers it, so the
    known dual is the octahedron with that one face replaced by the fan of
    three triangles around the seventh cell (7 vertices, 15 edges, 10
    triangles)."""
    m = I.icosphere(level)
    dirs = OCTA_DIRS / np.linalg.norm(OCTA_DIRS, axis=1, keepdims=True)
    seeds = np.array([int(np.argmax(m.V @ d)) for d in dirs], np.int32)
    ang = np.arccos(np.clip(m.V @ m.V[seeds].T, -1.0, 1.0))
    near = ang.min(1, keepdims=True)
    ptr, col, val = [0], [], []
    for v in range(m.n_v):
        cs = np.nonzero(ang[v] - near[v, 0] < delta)[0]
        w = np.where(ang[v, cs] == near[v, 0], 1.0, 0.6)
        col += [int(c) for c in cs]
        val += list(w / w.sum())
        ptr.append(len(col))
    U = (np.array(ptr, np.int64), np.array(col, np.int32), np.array(val, np.float64))
    expect = {(0, 2, 5), (0, 3, 4), (0, 3, 5), (1, 2, 4), (1, 2, 5), (1, 3, 4), (1, 3, 5),
              (0, 2, 6), (0, 4, 6), (2, 4, 6)}
    return m, seeds, U, expect, (0, 2, 4)
