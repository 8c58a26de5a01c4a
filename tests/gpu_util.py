"""Helpers for the GPU tests: decoding the Z layout on the host and locating
pairs in the packed triangle by counting (independent of the library)."""
import numpy as np


def packed_start(n: int) -> np.ndarray:
    """Offset of row i of the strict upper triangle, by counting row lengths."""
    length = (n - 1 - np.arange(n, dtype=np.int64))
    return np.concatenate([[0], np.cumsum(length)[:-1]])


def packed_pos(n: int, I, J) -> np.ndarray:
    I = np.asarray(I, dtype=np.int64)
    J = np.asarray(J, dtype=np.int64)
    return packed_start(n)[I] + (J - I - 1)


# The split layout of rows of at most two 128-byte chunks holds FP32 z (the
# rows the split arithmetic would not hold to 1e-5 are computed in FP32).
SPLIT_FP32_MAX_LPAD = 64


def split_is_fp32(zd) -> bool:
    return zd.mode == 1 and zd.l_pad <= SPLIT_FP32_MAX_LPAD


def bf16_to_f32(u16: np.ndarray) -> np.ndarray:
    return (u16.astype(np.uint32) << 16).view(np.float32)


def decode_z(zbytes: np.ndarray, zd) -> dict:
    """Host view of Z: dict with 'value' (FP64 n_pad x l_pad: what the tile
    kernels multiply, FP16 unscaled), plus 'hi'/'lo' for the split layout."""
    n_pad, l_pad, rb, mode = zd.n_pad, zd.l_pad, zd.row_bytes, zd.mode
    raw = np.asarray(zbytes, dtype=np.uint8)[: n_pad * rb].reshape(n_pad, rb)
    if mode == 0 or (mode == 1 and l_pad <= SPLIT_FP32_MAX_LPAD):  # FP32
        v = raw.view(np.float32).astype(np.float64)
        return {"value": v}
    if mode == 4:  # FP64
        return {"value": raw.view(np.float64).copy()}
    if mode == 2:  # BF16
        v = bf16_to_f32(raw.view(np.uint16)).astype(np.float64)
        return {"value": v}
    if mode == 3:  # FP16, stored as z * sqrt(l)
        v = raw.view(np.float16).astype(np.float64) / np.sqrt(zd.l)
        return {"value": v, "scaled": raw.view(np.float16).astype(np.float64)}
    # split: per 128-byte chunk, 32 hi then 32 lo
    u = raw.view(np.uint16).reshape(n_pad, l_pad // 32, 2, 32)
    hi = bf16_to_f32(u[:, :, 0, :].reshape(n_pad, l_pad)).astype(np.float64)
    lo = bf16_to_f32(u[:, :, 1, :].reshape(n_pad, l_pad)).astype(np.float64)
    return {"value": hi + lo, "hi": hi, "lo": lo}


def to_device(X, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(X))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()
