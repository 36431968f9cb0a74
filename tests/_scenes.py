"""Hand-built micro scenes for closed-form tests (inputs only, no renderer math)."""
import numpy as np

BOX_LO = np.array([-1.0, -1.0, 0.0])
BOX_HI = np.array([1.0, 1.0, 0.25])
DELTA = 0.25 / 512


def micro_scene(grid=(4, 4, 3), planes=(6, 6, 5), m=4, zmin=0.0, zmax=0.25, seed=None,
                std=0.5, mlp=None):
    """Scene dict in the layout of scenegen.make_scene.  Features are zero
    unless `seed` is given (then N(0, std)); occupancy is constant
    (zmin, zmax) unless arrays are passed."""
    lx, ly, lz = grid
    nx, ny, nz = planes
    rng = np.random.default_rng(seed) if seed is not None else None

    def arr(shape):
        if rng is None:
            return np.zeros(shape + (8,), np.float32)
        return (rng.standard_normal(shape + (8,)) * std).astype(np.float32)

    occ = np.empty((m, m, 2), np.float32)
    occ[..., 0] = zmin
    occ[..., 1] = zmax
    if mlp is None:
        mlp = np.zeros(499, np.float32) if rng is None else (rng.standard_normal(499) * 0.3).astype(np.float32)
    return dict(grid=arr((lz, ly, lx)), plane_xy=arr((ny, nx)), plane_xz=arr((nz, nx)),
                plane_yz=arr((nz, ny)), occ=occ, mlp=np.asarray(mlp, np.float32),
                box_lo=BOX_LO.copy(), box_hi=BOX_HI.copy())


def vertex_coords(n, lo, hi):
    return lo + np.arange(n) * (hi - lo) / (n - 1)
