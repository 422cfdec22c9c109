"""Host <-> device helpers shared by the GPU tests (no table arithmetic)."""
import numpy as np


def dev(a, bits=64):
    """numpy uint64 array -> contiguous int64 (bits=64) / int32 (bits=32) CUDA tensor."""
    import torch
    a = np.ascontiguousarray(a, dtype=np.uint64)
    if bits == 64:
        return torch.from_numpy(a.view(np.int64).copy()).cuda()
    return torch.from_numpy(a.astype(np.uint32).view(np.int32).copy()).cuda()


def host(t, bits=64):
    """CUDA int64/int32 tensor -> numpy uint64 array of the unsigned bit patterns."""
    a = t.detach().cpu().numpy()
    if bits == 64:
        return a.view(np.uint64).copy()
    return a.view(np.uint32).astype(np.uint64)


def u8(t):
    return t.detach().cpu().numpy().astype(np.uint8)


def image(table):
    """Raw table image copied to the host: (slots uint8, tags uint16 or None, locks uint64 words)."""
    r = table.raw()
    slots = r["slots"].cpu().numpy()
    tags = None if r["tags"] is None else r["tags"].cpu().numpy().view(np.uint16)
    locks32 = r["locks"].cpu().numpy().view(np.uint32)
    # the checker reads 64-bit lock words; pad to an even count
    if len(locks32) % 2:
        locks32 = np.concatenate([locks32, np.zeros(1, np.uint32)])
    return slots, tags, locks32.view(np.uint64)


def per_key_counts(keys, status, code):
    """dict key -> number of ops on that key whose status == code."""
    k = keys[status == code]
    u, c = np.unique(k, return_counts=True)
    return dict(zip(u.tolist(), c.tolist()))
