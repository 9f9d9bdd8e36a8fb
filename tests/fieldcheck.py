"""Shared helpers of the parity tests: per-field relative L2 and the one-step,
per-cell oracle check used at full lattice sizes."""
import numpy as np

FAMILIES_8 = {"rho": [0], "m": [1, 2, 3], "E": [4], "B": [5, 6, 7]}
FAMILIES_26 = dict(FAMILIES_8, G=list(range(8, 17)), H=list(range(17, 26)))


FAMILIES_5 = {"rho": [0], "m": [1, 2, 3], "E": [4]}
FAMILIES_9 = {"m": [0, 1, 2], "sigma_normal": [3, 4, 5], "sigma_shear": [6, 7, 8]}
FAMILIES_13 = {"rho": [0], "m": [1, 2], "E": [3], "B": [4, 5], "T": [6, 7, 8], "G": [9, 10, 11, 12]}


def families(K):
    return {26: FAMILIES_26, 5: FAMILIES_5, 9: FAMILIES_9, 13: FAMILIES_13}.get(K, FAMILIES_8)


def rel_l2(a, b, K):
    """Per field family: ||a - b||_2 / ||b||_2; vector families are normalised as
    vectors.  a, b: [K, N]."""
    a = np.asarray(a, np.float64).reshape(K, -1)
    b = np.asarray(b, np.float64).reshape(K, -1)
    out = {}
    for name, ks in families(K).items():
        num = np.sqrt(sum(np.sum((a[k] - b[k]) ** 2) for k in ks))
        den = np.sqrt(sum(np.sum(b[k] ** 2) for k in ks))
        out[name] = num / den if den > 0 else num
    return out


def upstream_cells(cells, shape, dim):
    """For each cell x and direction i, the linear index of x - e_i (periodic);
    returns [n, Q] (direction order 0, +x, -x, +y, -y, +z, -z)."""
    nx, ny, nz = shape
    cells = np.asarray(cells, np.int64)
    x = cells % nx
    y = (cells // nx) % ny
    z = cells // (nx * ny)
    NQ = 2 * dim + 1
    out = np.empty((len(cells), NQ), np.int64)
    out[:, 0] = cells
    for a in range(dim):
        for sgn, i in ((1, 2 * a + 1), (-1, 2 * a + 2)):
            c = [x.copy(), y.copy(), z.copy()]
            n = (nx, ny, nz)[a]
            c[a] = (c[a] - sgn) % n
            out[:, i] = c[0] + nx * (c[1] + ny * c[2])
    return out


def oracle_one_step(oracle, op, pre_gather, cells, shape, dim):
    """Expected post-step populations at `cells`: f_i(x) = collide(f(x - e_i))_i,
    from the pre-step populations returned by pre_gather(list of cells) -> [n, K, Q]."""
    up = upstream_cells(cells, shape, dim)
    uniq, inv = np.unique(up.ravel(), return_inverse=True)
    pre = pre_gather(uniq)
    post = oracle.collide_many(op, pre)
    NQ = 2 * dim + 1
    inv = inv.reshape(len(cells), NQ)
    K = pre.shape[1]
    out = np.empty((len(cells), K, NQ))
    for i in range(NQ):
        out[:, :, i] = post[inv[:, i], :, i]
    return out


def oracle_one_step_at(oracle, op, pre_gather, cells, shape, dim, t):
    """As oracle_one_step, with each upstream cell collided at its own coordinates and
    time t (the homogenized body's collision depends on where the cell is)."""
    up = upstream_cells(cells, shape, dim)
    uniq, inv = np.unique(up.ravel(), return_inverse=True)
    pre = pre_gather(uniq)
    nx, ny, _ = shape
    xyz = np.stack([uniq % nx, (uniq // nx) % ny, uniq // (nx * ny)], axis=1)
    post = oracle.collide_at(op, pre, xyz, t)
    NQ = 2 * dim + 1
    inv = inv.reshape(len(cells), NQ)
    K = pre.shape[1]
    out = np.empty((len(cells), K, NQ))
    for i in range(NQ):
        out[:, :, i] = post[inv[:, i], :, i]
    return out
