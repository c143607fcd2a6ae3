"""Shared helpers of the GPU parity tests: build matching oracle/GPU instances, compare faces.

Tolerance (floating point, FP64): the numerical flux of a face is a fixed linear combination of the
split characteristic values of its eight stencil cells, so its rounding error scales with the
physical fluxes entering it, not with its own (possibly cancelling) value. A face passes when
    ||Fhat_gpu - Fhat_oracle||_inf <= 1e-12 * max(||Fhat_oracle||_inf, S_face),
S_face = max over the face's eight stencil cells and components of |F(U_l)| (the physical flux in
the sweep direction). Faces whose selection differs are reported separately; they are accepted
only where the oracle's chi of a differing flag lies within 1e-9 (relative) of C_T.
"""
import numpy as np
import torch

from oracle import oracle as O
from oracle.census import (NEAR_CT, FaceCensus, census_text, cells_touched, near_bits,  # noqa: F401
                           trajectory_census)
from paper_1808_00037_amd import teno as T

REL_TOL = 1e-12
# chi of eq:norm goes through differences of neighbouring values (eq:smooth_expl) that cancel on
# smooth data, then through the power q: two evaluations that group the arithmetic differently agree
# to about 1e-11 absolute (measured at most 7.5e-12); the decisions themselves are compared bit for bit
CHI_TOL = 1e-10


def oracle_cfg(pr, scheme=O.TENO7X, eps=None, alpha_mode=0, ct=1e-5, C=1.0, q=6, characteristic=1):
    return O.Config(pr.sys, pr.nx, pr.ny, pr.x0, pr.x1, pr.y0, pr.y1, pr.bc_x, pr.bc_y, scheme=scheme,
                    alpha_mode=alpha_mode, gamma=pr.gamma, eps=eps, ct=ct, C=C, q=q,
                    characteristic=characteristic)


def solver_for(pr, dtype=torch.float64, scheme=T.TENO7X, eps=None, alpha_mode=0, ct=1e-5, C=1.0, q=6,
               characteristic=1):
    return T.Solver(pr.sys, pr.nx, pr.ny, pr.x0, pr.x1, pr.y0, pr.y1, pr.bc_x, pr.bc_y, dtype=dtype,
                    scheme=scheme, eps=eps, alpha_mode=alpha_mode, cfl=pr.cfl, gamma=pr.gamma, ct=ct,
                    C=C, q=q, characteristic=characteristic)


def _phys_flux_mag(sys, U, direction, gamma=1.4, adv=1.0):
    if sys == O.ADV1D:
        return np.abs(adv * U[0])
    if sys == O.BURGERS1D:
        return np.abs(0.5 * U[0] ** 2)
    if sys == O.EULER1D:
        rho, m, E = U
        u = m / rho
        p = (gamma - 1) * (E - 0.5 * rho * u * u)
        return np.max(np.abs(np.stack([m, m * u + p, u * (E + p)])), axis=0)
    rho, mx, my, E = U
    u, v = mx / rho, my / rho
    p = (gamma - 1) * (E - 0.5 * rho * (u * u + v * v))
    if direction == 0:
        F = np.stack([mx, mx * u + p, my * u, u * (E + p)])
    else:
        F = np.stack([my, mx * v, my * v + p, v * (E + p)])
    return np.max(np.abs(F), axis=0)


def face_scale(pr, U, direction):
    """S_face for every face of one direction: [ny, nx+1] (x) or [ny+1, nx] (y)."""
    s = _phys_flux_mag(pr.sys, U, direction, pr.gamma)
    mode = "wrap" if (pr.bc_x if direction == 0 else pr.bc_y) == O.PERIODIC else "edge"
    ax = 1 if direction == 0 else 0
    pad = [(0, 0), (0, 0)]
    pad[ax] = (4, 4)
    sp = np.pad(s, pad, mode=mode)
    n = s.shape[ax]
    out = None
    for k in range(8):       # face f reads cells f-4 .. f+3 = padded f .. f+7
        sl = [slice(None), slice(None)]
        sl[ax] = slice(k, k + n + 1)
        w = sp[tuple(sl)]
        out = w if out is None else np.maximum(out, w)
    return out


def compare_faces(pr, U_np, scheme=O.TENO7X, eps=None, alpha_mode=0, solver=None, ct=1e-5, C=1.0, q=6,
                  characteristic=1):
    """Run both sides on one state; return a report dict (asserting nothing). The GPU's chi of
    eq:norm is compared with the oracle's (chi_worst) and its own flags are checked against it
    (chi_flag_mismatch: a flag that disagrees with the GPU's chi away from rounding of C_T)."""
    opts = dict(scheme=scheme, eps=eps, alpha_mode=alpha_mode, ct=ct, C=C, q=q, characteristic=characteristic)
    cfg = oracle_cfg(pr, **opts)
    _, ex = O.rhs(cfg, U_np, want_faces=True)
    sv = solver or solver_for(pr, **opts)
    U = torch.from_numpy(np.ascontiguousarray(U_np)).cuda()
    g = sv.face_fluxes(U, chi=True)
    torch.cuda.synchronize()
    sv.poll()
    nfx = pr.ny * (pr.nx + 1)
    masks_g = g["masks"].cpu().numpy().view(np.uint32)
    flags_g = g["flags"].cpu().numpy().view(np.uint32)
    chi_g = g["chi"].double().cpu().numpy()
    rep = dict(alpha_gpu=g["alpha"].cpu().numpy(), alpha_orc=ex["alpha"], nfaces=0, worst=0.0, flips=0,
               flips_near_ct=0, flag_diffs=0, chi_worst=0.0, chi_flag_mismatch=0)
    nbits = 6 * np.asarray(U_np).shape[0]
    dirs = [("x", 0, g["Fx"], ex["Fx"], ex["masks_x"], ex["flags_x"], ex["chi_x"], slice(0, nfx))]
    if pr.sys == O.EULER2D:
        dirs.append(("y", 1, g["Fy"], ex["Fy"], ex["masks_y"], ex["flags_y"], ex["chi_y"], slice(nfx, None)))
    for name, d, Fg, Fo, mo, fo, chi, sec in dirs:
        Fg = Fg.cpu().numpy()
        mg = masks_g[sec].reshape(mo.shape)
        fg = flags_g[sec].reshape(fo.shape)
        cg = chi_g[sec].reshape(chi.shape)
        rep["chi_worst"] = max(rep["chi_worst"], float(np.abs(cg[..., :nbits] - chi[..., :nbits]).max()))
        # the GPU's flags follow its own chi (a decision within rounding of C_T may go either way)
        bits = ((fg[..., None] >> np.arange(nbits, dtype=np.uint32)) & 1).astype(bool)
        own = cg[..., :nbits] >= ct
        rep["chi_flag_mismatch"] += int(np.count_nonzero((bits != own) & (np.abs(cg[..., :nbits] / ct - 1) >= NEAR_CT)))
        same = mg == mo
        # flags: every difference must sit within rounding of the cut-off
        fdiff = fg != fo
        rep["flag_diffs"] += int(fdiff.sum())
        for idx in np.argwhere(fdiff):
            x = int(fg[tuple(idx)] ^ fo[tuple(idx)])
            bits = [b for b in range(24) if (x >> b) & 1]   # bit 6s+3side+k <-> chi[..., 6s+3side+k]
            if all(abs(chi[tuple(idx)][b] / ct - 1.0) < 1e-9 for b in bits):
                rep["flips_near_ct"] += 1
        # masks are a function of the flags of a face and its two neighbours along the line
        ax = 1 if d == 0 else 0
        near = fdiff.copy()
        near |= np.roll(fdiff, 1, axis=ax) | np.roll(fdiff, -1, axis=ax)
        rep["flips"] += int((~same).sum())
        rep["mask_diffs_unexplained"] = rep.get("mask_diffs_unexplained", 0) + int((~same & ~near).sum())
        scale = np.maximum(np.max(np.abs(Fo), axis=0), face_scale(pr, U_np, d))
        err = np.max(np.abs(Fg - Fo), axis=0) / scale
        err = np.where(same, err, 0.0)
        rep["nfaces"] += err.size
        rep["worst"] = max(rep["worst"], float(err.max()))
        rep[f"worst_{name}"] = float(err.max())
    return rep


def census_line(rep):
    """One line of the selection census of a face comparison."""
    return (f"faces {rep['nfaces']}, flag words differing {rep['flag_diffs']} (within rounding of C_T: "
            f"{rep['flips_near_ct']}), mask words differing {rep['flips']} (unexplained: "
            f"{rep.get('mask_diffs_unexplained', 0)}), worst face error {rep['worst']:.2e}")


def assert_face_parity(rep):
    print("[census]", census_line(rep), f"chi difference {rep['chi_worst']:.1e}", flush=True)
    assert rep["flag_diffs"] == rep["flips_near_ct"], rep
    assert rep["chi_worst"] <= CHI_TOL and rep["chi_flag_mismatch"] == 0, rep
    assert rep.get("mask_diffs_unexplained", 0) == 0, rep
    assert rep["worst"] <= REL_TOL, rep
    assert np.allclose(rep["alpha_gpu"], rep["alpha_orc"], rtol=1e-14, atol=0), rep


