"""GPU-versus-oracle comparison helpers.

Pass criterion for a traced frame (floating point): on at least 99.9% of
pixels the object id is identical and the hit point lies within a
Euclidean distance of 1e-3 scene units of the oracle's (misses compare their
final positions the same way).  The remaining 0.1% covers rays whose fate is decided by a
rounding-level difference: grazing hits and silhouettes, where FP32 and FP64
legitimately disagree.
"""
import numpy as np

HIT_TOL = 1e-3
FRAC = 0.999


def compare(gpu, ref, idx=None, hit_tol=HIT_TOL):
    """gpu: dict of numpy arrays for the whole frame; ref: oracle dict for
    the pixels `idx` (all pixels if None)."""
    g = {k: (v if idx is None else v[idx]) for k, v in gpu.items() if v is not None and not k.startswith("_")}
    same = g["id"] == ref["id"]
    err = np.linalg.norm(g["hit"].astype(np.float64) - ref["hit"], axis=1)
    ok = same & (err <= hit_tol)
    both = same & (ref["id"] >= 0)
    rep = dict(n=int(len(ok)), frac_ok=float(ok.mean()), frac_id=float(same.mean()),
               max_hit_err=float(err[same].max()) if same.any() else 0.0,
               p999_hit_err=float(np.quantile(err[same], 0.999)) if same.any() else 0.0,
               max_t_err=float(np.abs(g["t"] - ref["t"])[both].max()) if both.any() else 0.0,
               max_dir_err=float(np.abs(g["dir"] - ref["dir"]).max(axis=1)[both].max()) if both.any() else 0.0,
               hits=float((ref["id"] >= 0).mean()))
    return rep


def assert_parity(rep, frac=FRAC):
    assert rep["frac_ok"] >= frac, rep
