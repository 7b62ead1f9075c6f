"""Host-side readers of the documented tiled-matrix layout (include/gpr.h), for tests."""
import numpy as np


def tiles_to_dense_lower(raw: np.ndarray, n: int, b: int, esize: int) -> np.ndarray:
    """Dense lower matrix of T b rows, T = ceil(n / b), from the bytes of a K_tiles buffer
    (regions D and O); n x n when b divides n, else including the identity padding."""
    T = -(-n // b)
    L = np.zeros((T * b, T * b), dtype=np.float64)
    dreg = raw[: T * b * b * 8].view(np.float64)
    for k in range(T):
        L[k * b:(k + 1) * b, k * b:(k + 1) * b] = np.tril(dreg[k * b * b:(k + 1) * b * b].reshape(b, b))
    off0 = 2 * T * b * b * 8
    dt = np.float64 if esize == 8 else np.float32
    oreg = raw[off0:].view(dt)
    for j in range(T):
        for i in range(j + 1, T):
            idx = j * (T - 1) - j * (j - 1) // 2 + (i - j - 1)
            L[i * b:(i + 1) * b, j * b:(j + 1) * b] = oreg[idx * b * b:(idx + 1) * b * b].reshape(b, b)
    return L


def winv_tiles(raw: np.ndarray, n: int, b: int):
    T = -(-n // b)
    wreg = raw[T * b * b * 8: 2 * T * b * b * 8].view(np.float64)
    return [wreg[k * b * b:(k + 1) * b * b].reshape(b, b) for k in range(T)]


def diag_tile_offset_bytes(k: int, b: int) -> int:
    return k * b * b * 8


def lower_row(buf, n: int, b: int, esize: int, i: int) -> np.ndarray:
    """Row i (entries 0..i) of the lower factor held in a K_tiles buffer, reading only that
    row's bytes; `buf` is the buffer as a flat uint8 torch tensor (device or host)."""
    T = -(-n // b)
    I, r = divmod(i, b)
    parts = []
    off0 = 2 * T * b * b * 8
    dt = np.float64 if esize == 8 else np.float32
    for J in range(I):
        idx = J * (T - 1) - J * (J - 1) // 2 + (I - J - 1)
        start = off0 + (idx * b * b + r * b) * esize
        parts.append(buf[start:start + b * esize].cpu().numpy().view(dt).astype(np.float64))
    start = (I * b * b + r * b) * 8
    parts.append(buf[start:start + (r + 1) * 8].cpu().numpy().view(np.float64))
    return np.concatenate(parts)
