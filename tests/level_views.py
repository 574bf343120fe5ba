"""Host-side construction of level views (cell lists) for tests."""
import numpy as np


def _map(i, n, bc):
    return np.mod(i, n) if bc == "periodic" else np.clip(i, 0, n - 1)


def mesh_level_view(shape, M, bcs, cells=None):
    """Level view of (a subset of) a uniform mesh.

    shape: cells per axis (x first); cells: [C, d] updated cells (default: all).
    Returns numpy arrays (pred_cells, pred_patch, upd, upd_nbr) in the layout of
    ader_step_level: predicted = updated cells + their face neighbours.
    """
    d = len(shape)
    strides = [1] + list(np.cumprod(shape[:-1]))
    lin = lambda c: int(sum(int(c[k]) * strides[k] for k in range(d)))
    if cells is None:
        grids = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
        cells = np.stack([g.ravel(order="F") for g in grids], axis=1)
    cells = np.asarray(cells)
    pred = {}
    order = []

    def add(c):
        key = tuple(int(x) for x in c)
        if key not in pred:
            pred[key] = len(order)
            order.append(key)
        return pred[key]
    upd = [add(c) for c in cells]
    nbr = []
    for c in cells:
        row = []
        for k in range(d):
            for sgn in (-1, 1):
                raw = int(c[k]) + sgn
                if bcs[k] != "periodic" and (raw < 0 or raw >= shape[k]):
                    row.append(-1)
                    continue
                cc = list(c)
                cc[k] = _map(raw, shape[k], bcs[k])
                row.append(add(cc))
        nbr.append(row)
    S = 2 * M + 1
    offs = np.arange(-M, M + 1)
    patches = []
    for key in order:
        idx = np.zeros((S,) * d, dtype=np.int64)
        for o in np.ndindex(*((S,) * d)):
            cc = [_map(key[k] + offs[o[k]], shape[k], bcs[k]) for k in range(d)]
            idx[o] = lin(cc)
        patches.append(idx.transpose(tuple(range(d - 1, -1, -1))).ravel())  # x fastest
    pred_cells = np.array([lin(k) for k in order], dtype=np.int32)
    return (pred_cells, np.concatenate(patches).astype(np.int32),
            np.array(upd, dtype=np.int32), np.array(nbr, dtype=np.int32).ravel())
