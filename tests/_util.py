"""Helpers shared by the tests: record decoding, device upload, tolerances."""
import numpy as np

REC_DTYPE = np.dtype([("mx", "<f8"), ("my", "<f8"), ("l11", "<f4"), ("l21", "<f4"), ("l22", "<f4"), ("cr", "<f4"),
                      ("cg", "<f4"), ("cb", "<f4"), ("o", "<f4"), ("inv_nu", "<f4"), ("nb", "<f4"), ("hs", "<f4"),
                      ("entry", "<u4"), ("ey", "<f4")])
assert REC_DTYPE.itemsize == 64

PARAMS = ("means", "scales", "quats", "nu", "opacity", "sh")


def decode_records(raw: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(raw).view(REC_DTYPE).reshape(-1)


def make_projected(sss, records, keys, rect, touched, ell, device="cuda"):
    """Projected entries built on the host: the 128-byte line of each entry
    holds the 64-byte record, the FP64 ellipse and the int16 rectangle."""
    import torch
    E = records.shape[0]
    ent = np.zeros((E, 128), np.uint8)
    ent[:, :64] = records
    ent[:, 64:96] = np.ascontiguousarray(ell, np.float64).view(np.uint8).reshape(E, 32)
    ent[:, 96:104] = np.ascontiguousarray(rect, np.int16).view(np.uint8).reshape(E, 8)
    return sss.Projected(torch.as_tensor(ent, device=device),
                         torch.as_tensor(np.ascontiguousarray(keys, np.uint32).view(np.int32), device=device),
                         torch.as_tensor(np.ascontiguousarray(touched, np.int32), device=device))


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


def pure_rel_fraction(got, ref, rel=1e-3, mask=None, tiny=1e-30):
    """Fraction of elements (rows in mask) with |got - ref| <= rel |ref|: the
    plain relative criterion, without the per-array rms floor of
    grad_close (reported beside it)."""
    got = np.asarray(got, np.float64).reshape(got.shape[0], -1)
    ref = np.asarray(ref, np.float64).reshape(ref.shape[0], -1)
    ok = np.abs(got - ref) <= rel * np.abs(ref) + tiny
    if mask is not None:
        ok = ok[mask]
    return float(ok.mean()) if ok.size else 1.0

