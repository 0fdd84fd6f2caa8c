"""Helpers shared by the tests: record decoding, device upload, tolerances."""
import numpy as np

REC_DTYPE = np.dtype([("mx", "<f8"), ("my", "<f8"), ("qa", "<f4"), ("qb", "<f4"), ("qc", "<f4"), ("cr", "<f4"),
                      ("cg", "<f4"), ("cb", "<f4"), ("o", "<f4"), ("inv_nu", "<f4"), ("nb", "<f4"), ("hs", "<f4"),
                      ("entry", "<u4"), ("ey", "<f4")])
assert REC_DTYPE.itemsize == 64

PARAMS = ("means", "scales", "quats", "nu", "opacity", "sh")


def decode_records(raw: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(raw).view(REC_DTYPE).reshape(-1)


def to_device(scene, device="cuda"):
    import torch
    out = {k: torch.as_tensor(np.ascontiguousarray(scene[k]), dtype=torch.float32, device=device)
           for k in PARAMS}
    out["sh_degree"] = int(scene["sh_degree"])
    return out


def grad_close(got, ref, rel=1e-3, mask=None):
    """|got - ref| <= rel * max(|ref|, rms(ref)) elementwise; returns (ok, worst ratio)."""
    got = np.asarray(got, np.float64).reshape(got.shape[0], -1)
    ref = np.asarray(ref, np.float64).reshape(ref.shape[0], -1)
    rms = np.sqrt(np.mean(ref ** 2)) if ref.size else 0.0
    tol = rel * np.maximum(np.abs(ref), rms) + 1e-30
    ratio = np.abs(got - ref) / tol
    if mask is not None:
        ratio = ratio[mask]
    worst = float(ratio.max()) if ratio.size else 0.0
    return worst <= 1.0, worst
