"""Helpers shared by the GPU tests (no method arithmetic here)."""
import numpy as np


def codes_to_set(codes):
    return set(int(c) for c in np.asarray(codes, dtype=np.uint64).tolist())


def pairs_to_codes(pairs):
    p = np.asarray(pairs, dtype=np.uint64).reshape(-1, 2)
    return (p[:, 0] << np.uint64(32)) | p[:, 1]


def to_device(col):
    import torch
    chars = torch.from_numpy(col.chars.copy()).cuda() if col.chars.size else \
        torch.zeros(0, dtype=torch.uint8, device="cuda")
    offs = torch.from_numpy(col.offsets.astype(np.int64)).cuda()
    return chars, offs
