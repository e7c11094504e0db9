"""Comparison helpers for GPU-vs-oracle parity tests.

States live on a surface, so their 6x6 covariance has rank 5: the position
variance along the surface normal is zero up to rounding.  Covariances are
therefore compared on the five free parameters (u, v, k, phi, theta), u and v
the local surface coordinates (barrel: r*phi direction and z; disk: r*phi
direction and r), element-wise to a fraction of sqrt(C_ii C_jj); the normal
variance is checked separately against the position variances.
"""
import numpy as np

from oracle import KAPPA_1E4, candidate_conditioning, update_conditioning  # noqa: F401

BARREL = 0
PARAM_FLOORS = np.array([1.0, 1.0, 1.0, 0.0, 1.0, 1.0])  # cm, cm, cm, -, rad, rad


def wrap(a):
    return (a + np.pi) % (2 * np.pi) - np.pi


def param_rel(pg, po):
    """|delta p_i| / max(|p_i|, floor_i) (phi difference wrapped); equal
    values compare as 0 (k = 0 exactly without a field)."""
    d = pg - po
    d[:, 4] = wrap(d[:, 4])
    den = np.maximum(np.abs(po), PARAM_FLOORS)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(d == 0.0, 0.0, np.abs(d) / den)


def chi2_tol(c2o):
    """Bound on |chi2_GPU - chi2_oracle| for a track chi2: 1e-3 absolute, or
    one float32 ulp of the value where that is coarser (chi2 >= 8192): the
    GPU returns the chi2 as float32, which cannot hold it closer."""
    c = np.abs(np.asarray(c2o, dtype=np.float64))
    return np.maximum(1e-3, np.spacing(c.astype(np.float32)).astype(np.float64))


def local_frame_T(p, kinds):
    """5x6 maps from (x, y, z, k, phi, theta) to (u, v, k, phi, theta)."""
    n = p.shape[0]
    r = np.hypot(p[:, 0], p[:, 1])
    c, s = p[:, 0] / r, p[:, 1] / r
    T = np.zeros((n, 5, 6))
    T[:, 0, 0], T[:, 0, 1] = -s, c
    bar = kinds == BARREL
    T[bar, 1, 2] = 1.0
    T[~bar, 1, 0], T[~bar, 1, 1] = c[~bar], s[~bar]
    T[:, 2, 3] = T[:, 3, 4] = T[:, 4, 5] = 1.0
    nrm = np.zeros((n, 3))
    nrm[bar, 0], nrm[bar, 1] = c[bar], s[bar]
    nrm[~bar, 2] = 1.0
    return T, nrm


def cov_rel(Cg, Co, p, kinds):
    """Per state: max |dC5_ij| / sqrt(C5_ii C5_jj) on the surface parameters,
    and the normal variances (GPU, oracle) relative to the largest position
    variance."""
    T, nrm = local_frame_T(p, kinds)
    Cg5 = T @ Cg @ T.transpose(0, 2, 1)
    Co5 = T @ Co @ T.transpose(0, 2, 1)
    d = np.sqrt(np.abs(np.einsum("nii->ni", Co5)))
    rel = np.abs(Cg5 - Co5) / (d[:, :, None] * d[:, None, :] + 1e-300)
    scale = np.max(np.einsum("nii->ni", Co[:, :3, :3]), axis=1)
    ng = np.abs(np.einsum("ni,nij,nj->n", nrm, Cg[:, :3, :3], nrm)) / scale
    no = np.abs(np.einsum("ni,nij,nj->n", nrm, Co[:, :3, :3], nrm)) / scale
    return rel.max(axis=(1, 2)), ng, no


def check_identical_candidates(rel, kappa, dchi2, tag=""):
    """Parity of building candidates whose hit lists equal the oracle's:
    every one within max(1e-4, 2^-24 kappa) in the parameters, and the
    well-conditioned ones (kappa <= KAPPA_1E4) within 1e-3 in the chi2 sum.
    Prints the counts and the spread of the ill-conditioned ones."""
    rel, kappa, dchi2 = (np.asarray(a, dtype=np.float64) for a in (rel, kappa, dchi2))
    kap = np.where(np.isnan(kappa), np.inf, kappa)
    bound = np.maximum(1e-4, 2.0 ** -24 * kap)
    ill = kap > KAPPA_1E4
    well = ~ill
    msg = (f"{tag}identical candidates {rel.size}: well-conditioned {well.sum()} (params max "
           f"{rel[well].max() if well.any() else 0:.3g}, chi2 max {dchi2[well].max() if well.any() else 0:.3g}); "
           f"ill-conditioned {ill.sum()} (params max {rel[ill].max() if ill.any() else 0:.3g}, p99 "
           f"{np.percentile(rel[ill], 99) if ill.any() else 0:.3g})")
    print(msg, flush=True)
    assert np.all(rel <= bound), msg
    assert np.all(dchi2[well] <= 1e-3), msg
    return msg
