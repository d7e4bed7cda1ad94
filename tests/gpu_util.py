"""Host <-> device helpers for the GPU tests (moves bytes through signed views so that only the
barest tensor operations touch the unsigned dtypes)."""
import numpy as np
import torch

_SIGNED = {np.dtype(np.uint8): (np.uint8, torch.uint8), np.dtype(np.uint16): (np.int16, torch.int16),
           np.dtype(np.uint32): (np.int32, torch.int32), np.dtype(np.uint64): (np.int64, torch.int64)}
_UNSIGNED_T = {torch.int16: torch.uint16, torch.int32: torch.uint32, torch.int64: torch.uint64,
               torch.uint8: torch.uint8}
_SIGNED_T = {torch.uint16: torch.int16, torch.uint32: torch.int32, torch.uint64: torch.int64,
             torch.uint8: torch.uint8, torch.float64: torch.float64}


def to_device(a: np.ndarray, device="cuda:0") -> torch.Tensor:
    """numpy unsigned array -> device tensor of the same unsigned dtype (contiguous)."""
    a = np.ascontiguousarray(a)
    np_s, t_s = _SIGNED[a.dtype]
    t = torch.from_numpy(a.view(np_s)).to(device)
    return t.view(_UNSIGNED_T[t_s]) if t_s != torch.uint8 else t


def to_host(t: torch.Tensor) -> np.ndarray:
    """device tensor (any strides) -> numpy array of the matching unsigned / float dtype."""
    s = t.view(_SIGNED_T[t.dtype]).cpu().numpy()
    if t.dtype == torch.uint16:
        return s.view(np.uint16)
    if t.dtype == torch.uint32:
        return s.view(np.uint32)
    if t.dtype == torch.uint64:
        return s.view(np.uint64)
    return s


def padded_image(a: np.ndarray, pitch: int, offset: int, device="cuda:0") -> torch.Tensor:
    """Device view of `a` inside a wider buffer: row pitch `pitch` elements, first pixel at
    element `offset` (so the base may be misaligned)."""
    H, W = a.shape
    buf = np.zeros((H + 1) * pitch + offset, a.dtype)
    view = np.lib.stride_tricks.as_strided(buf[offset:], shape=(H, W), strides=(pitch * a.itemsize, a.itemsize))
    view[...] = a
    dev = to_device(buf, device)
    return dev[offset:offset + H * pitch].view(H, pitch)[:, :W] if offset + H * pitch <= buf.size else None
