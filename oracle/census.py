"""Selection census: the oracle's per-face selection compared with another implementation's words.

TEST INFRASTRUCTURE, like the rest of oracle/: used by the test-suite and the CPU leg of the
benchmark only. It holds no scheme arithmetic; it compares words and reads the oracle's chi.

A cut-off decision (eq:seclect) whose chi lies within NEAR_CT (relative) of C_T may go either way
between two implementations that round differently; every other flag must agree, and a mask word
(Table 3 applied to the neighbour vector of eq:vec) may differ only where such a decision of the
face or of a neighbour face along its line is involved.
"""
import numpy as np

from . import oracle as O

NEAR_CT = 1e-9      # a cut-off decision within this relative distance of C_T may go either way


def near_bits(chi, ct):
    """Per face, a 24-bit word with bit 6s+3side+k set where chi of that decision lies within
    rounding (NEAR_CT, relative) of C_T. chi: [..., 24]."""
    near = np.abs(chi / ct - 1.0) < NEAR_CT
    w = np.zeros(chi.shape[:-1], dtype=np.uint32)
    for b in range(chi.shape[-1]):
        w |= near[..., b].astype(np.uint32) << np.uint32(b)
    return w


class FaceCensus:
    """The oracle's selection of every face of a 2D state, gathered strip by strip (masks, flags,
    which decisions sit within rounding of C_T, optionally the face fluxes), then compared with the
    GPU's words:
      * a flag bit may differ only where the oracle's chi of that decision is near C_T;
      * a mask word may differ only where a flag of the face or of a neighbour face along the line
        (the faces eq:vec reads) is near C_T."""

    def __init__(self, pr, ct=1e-5, keep_flux=False):
        ny, nx = pr.ny, pr.nx
        self.pr, self.ct = pr, ct
        self.mx = np.zeros((ny, nx + 1), np.uint32)
        self.my = np.zeros((ny + 1, nx), np.uint32)
        self.fx = np.zeros_like(self.mx)
        self.fy = np.zeros_like(self.my)
        self.nx_ = np.zeros_like(self.mx)
        self.ny_ = np.zeros_like(self.my)
        nv = pr.U0.shape[0]
        self.Fx = np.zeros((nv, ny, nx + 1)) if keep_flux else None
        self.Fy = np.zeros((nv, ny + 1, nx)) if keep_flux else None

    def on_faces(self, j0, j1, f):
        fy = f["masks_y"].shape[0]
        self.mx[j0:j1] = f["masks_x"]
        self.fx[j0:j1] = f["flags_x"]
        self.nx_[j0:j1] = near_bits(f["chi_x"], self.ct)
        self.my[j0:j0 + fy] = f["masks_y"]
        self.fy[j0:j0 + fy] = f["flags_y"]
        self.ny_[j0:j0 + fy] = near_bits(f["chi_y"], self.ct)
        if self.Fx is not None:
            self.Fx[:, j0:j1] = f["Fx"]
            self.Fy[:, j0:j0 + fy] = f["Fy"]

    def compare(self, masks_g, flags_g=None):
        """masks_g/flags_g: the GPU's words of every face (x-faces then y-faces, uint32)."""
        nfx = self.mx.size
        rep = dict(faces=nfx + self.my.size, flag_diffs=0, flag_diffs_unexplained=0, mask_diffs=0,
                   mask_diffs_unexplained=0)
        diffs = {}
        for d, (mo, fo, nb) in enumerate(((self.mx, self.fx, self.nx_), (self.my, self.fy, self.ny_))):
            sec = slice(0, nfx) if d == 0 else slice(nfx, None)
            mg = masks_g[sec].reshape(mo.shape)
            if flags_g is not None:
                fg = flags_g[sec].reshape(fo.shape)
                x = fg ^ fo
                rep["flag_diffs"] += int(np.count_nonzero(x))
                rep["flag_diffs_unexplained"] += int(np.count_nonzero(x & ~nb))
            md = mg != mo
            ax = 1 if d == 0 else 0
            near = nb != 0
            near_line = near.copy()
            if ax == 1:
                near_line[:, 1:] |= near[:, :-1]
                near_line[:, :-1] |= near[:, 1:]
            else:
                near_line[1:] |= near[:-1]
                near_line[:-1] |= near[1:]
            rep["mask_diffs"] += int(np.count_nonzero(md))
            rep["mask_diffs_unexplained"] += int(np.count_nonzero(md & ~near_line))
            diffs[d] = md
        rep["near_ct_faces"] = int(np.count_nonzero(self.nx_) + np.count_nonzero(self.ny_))
        return rep, diffs


def census_text(rep):
    return (f"faces {rep['faces']}, decisions near C_T {rep['near_ct_faces']}, flag words differing "
            f"{rep['flag_diffs']} (unexplained {rep['flag_diffs_unexplained']}), mask words differing "
            f"{rep['mask_diffs']} (unexplained {rep['mask_diffs_unexplained']})")


def cells_touched(diffs, shape, radius, periodic):
    """Cells whose value a differing selection at these faces can reach within `radius` more cells
    along rows and columns (x-face f of a row touches cells f-1 and f; y-face likewise)."""
    from scipy import ndimage
    ny, nx = shape
    hit = np.zeros(shape, bool)
    mx, my = diffs[0], diffs[1]
    hit[:, :] |= mx[:, :nx] | mx[:, 1:]           # cells right and left of each x-face
    hit[:, :] |= my[:ny, :] | my[1:, :]
    if radius > 0 and hit.any():
        hit = ndimage.maximum_filter(hit.astype(np.uint8), size=2 * radius + 1,
                                     mode="wrap" if periodic else "nearest").astype(bool)
    return hit


def _near_line(nb, ax):
    near = nb != 0
    out = near.copy()
    if ax == 1:
        out[:, 1:] |= near[:, :-1]
        out[:, :-1] |= near[:, 1:]
    else:
        out[1:] |= near[:-1]
        out[:-1] |= near[1:]
    return out


def trajectory_census(pr, cfg, U0, nsteps, gpu_masks=None, dt=0.0):
    """The oracle's SSP-RK3 trajectory taken stage by stage (oracle.step_stages, bitwise its run())
    with every face's selection in view. gpu_masks ([nsteps, 3, nfaces] words recorded by the GPU)
    are compared face by face: a differing word is explained when a cut-off decision of the face or
    of a neighbour face along its line lies within rounding of C_T, or when an earlier stage already
    differed (its state then differs too). Returns (final state, alpha [nsteps, 3, 8], dt [nsteps],
    census dict)."""
    U = np.ascontiguousarray(U0, dtype=np.float64).copy()
    alphas, dts = [], []
    rep = dict(words=0, mask_diffs=0, unexplained=0, downstream=0, near_ct_faces=0)
    diverged = False
    two_d = pr.sys == O.EULER2D
    for n in range(nsteps):
        faces = []
        U, info = O.step_stages(cfg, U, dt=dt, cfl=pr.cfl, on_faces=lambda s, j0, j1, f: faces.append(f))
        alphas.append(info["alpha"])
        dts.append(info["dt"])
        if gpu_masks is None:
            continue
        for s, f in enumerate(faces):
            parts = [("x", f["masks_x"], near_bits(f["chi_x"], cfg.ct), 1)]
            if two_d:
                parts.append(("y", f["masks_y"], near_bits(f["chi_y"], cfg.ct), 0))
            off = 0
            for _, mo, nb, ax in parts:
                mg = np.asarray(gpu_masks[n, s, off:off + mo.size]).view(np.uint32).reshape(mo.shape)
                off += mo.size
                md = mg != mo
                nd = int(np.count_nonzero(md))
                rep["words"] += mo.size
                rep["mask_diffs"] += nd
                rep["near_ct_faces"] += int(np.count_nonzero(nb))
                if nd:
                    bad = int(np.count_nonzero(md & ~_near_line(nb, ax)))
                    if diverged:
                        rep["downstream"] += bad
                    else:
                        rep["unexplained"] += bad
            if rep["mask_diffs"]:
                diverged = True
    return U, np.array(alphas), np.array(dts), rep
