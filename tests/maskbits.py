"""Host-side packing of prior masks into the library's bitmask layout for the
tests: bit e (least significant first) of 32-bit word e // 32 is sample e."""
import numpy as np


def pack_bits(mask) -> np.ndarray:
    """bool/uint8 [S] -> int32 [ceil(S/32)] words."""
    m = np.asarray(mask).reshape(-1) != 0
    by = np.packbits(m, bitorder="little")
    pad = (-by.size) % 4
    if pad:
        by = np.concatenate([by, np.zeros(pad, dtype=np.uint8)])
    return by.view("<u4").astype(np.uint32).view(np.int32)


def unpack_bits(words, S: int) -> np.ndarray:
    """int32 [ceil(S/32)] words -> bool [S]."""
    by = np.ascontiguousarray(np.asarray(words).astype(np.int32)).view("<u4").view(np.uint8)
    return np.unpackbits(by, bitorder="little")[:S].astype(bool)
