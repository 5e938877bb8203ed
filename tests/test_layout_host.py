"""The xy4 storage order on the host: the Python views of the records (used by the GPU tests to
inspect and rewrite grids) against a NumPy model written from the layout's definition.

Records are stored as [t][z/2][y/2][x][z&1][y&1] with x rounded up to even and y, z rounded up to
even, so that a 128-byte line holds the 2 x 2 x 2 records of an x pair; padding records are zero.
"""
import numpy as np
import torch

from paper_2304_09953_amd import dock, inputs as I, pipeline as P


def storage_model(rec):
    """[t][z][y][x][4] records -> flat storage, each record at the byte offset the layout defines."""
    T, nz, ny, nx, _ = rec.shape
    nxp, nby, nbz = (nx + 1) // 2 * 2, (ny + 1) // 2, (nz + 1) // 2
    type_floats = 16 * nxp * nby * nbz
    out = np.zeros(T * type_floats, np.float32)
    for t in range(T):
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    byte = 64 * (x + nxp * (y // 2 + nby * (z // 2))) + 16 * (y % 2 + 2 * (z % 2))
                    at = t * type_floats + byte // 4
                    out[at:at + 4] = rec[t, z, y, x]
    return out


def _host_pocket(dims, n_types, grids):
    dp = P.DevicePocket.__new__(P.DevicePocket)
    dp.pocket = I.make_pocket(dims, n_types, n_prot=10)
    dp.layout = dock.LAYOUT_XY4
    dp.grids = grids
    return dp


def test_records_views_invert_the_storage_order():
    rng = np.random.default_rng(1)
    for dims in ((6, 5, 7), (7, 4, 10), (4, 3, 4), (5, 2, 2)):
        nx, ny, nz = dims
        rec = rng.normal(size=(2, nz, ny, nx, 4)).astype(np.float32)
        flat = storage_model(rec)
        dp = _host_pocket(dims, 2, torch.from_numpy(flat.copy()))
        assert torch.equal(dp.records(), torch.from_numpy(rec)), dims
        back = _host_pocket(dims, 2, torch.full_like(dp.grids, 7.0))
        back.write_records(torch.from_numpy(rec))
        assert torch.equal(back.grids, torch.from_numpy(flat)), dims


def test_grid_bytes_follow_the_layout():
    for dims in ((6, 5, 7), (7, 4, 10), (96, 96, 96)):
        nx, ny, nz = dims
        g = dock.grid_desc(I.make_pocket(dims, 3, n_prot=10), layout=dock.LAYOUT_XY4)
        assert dock.grid_bytes(g) == 3 * 128 * ((nx + 1) // 2) * ((ny + 1) // 2) * ((nz + 1) // 2)
