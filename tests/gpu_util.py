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


def held_lock_bitmap(lock_words32, num_buckets, stride=1):
    """Lock array (byte b * stride: bucket b, nonzero while held) -> the
    layout checker's bitmap of held locks (bit b % 64 of 64-bit word b // 64)."""
    by = np.ascontiguousarray(lock_words32, dtype=np.uint32).view(np.uint8)[::stride][:num_buckets]
    packed = np.packbits(by != 0, bitorder="little")
    packed = np.concatenate([packed, np.zeros(-len(packed) % 8, np.uint8)])
    return packed.view(np.uint64)


def busy_lock_queues(table):
    """Number of lock queues with a ticket not yet served (next != serving)."""
    q = table.raw()["lock_queues"].cpu().numpy().view(np.uint64)
    return int(((q >> np.uint64(32)) != (q & np.uint64(0xFFFFFFFF))).sum())


def image(table):
    """Raw table image copied to the host: (slots uint8, tags uint16 or None,
    bitmap of held bucket locks as uint64 words)."""
    r = table.raw()
    slots = r["slots"].cpu().numpy()
    tags = None if r["tags"] is None else r["tags"].cpu().numpy().view(np.uint16)
    return slots, tags, held_lock_bitmap(r["locks"].cpu().numpy().view(np.uint32), table.num_buckets,
                                         r["lock_stride"])


def per_key_counts(keys, status, code):
    """dict key -> number of ops on that key whose status == code."""
    k = keys[status == code]
    u, c = np.unique(k, return_counts=True)
    return dict(zip(u.tolist(), c.tolist()))


def full_is_genuine(t, full_keys):
    """A two-choice table reports FULL only when both candidate buckets are full,
    iceberg only when its front bucket and both backyard choices are: checked on
    the final image of an insert-only table, with the oracle's own placement
    rules for the candidate buckets."""
    import oracle
    slots, tags, _ = image(t)
    if t.kv_bits == 64:
        kw = slots.view(np.uint64)[0::2]
        free = kw >= np.uint64((1 << 64) - 2)
    else:
        kw = slots.view(np.uint32)[0::2]
        free = kw >= np.uint32(0xFFFFFFFE)
    occ = (~free).reshape(t.num_buckets, t.bucket_slots).sum(axis=1)
    for k in np.unique(full_keys).tolist():
        if t.design.startswith("ICEBERG"):
            cand = oracle.iceberg_buckets(k, t.num_buckets)
        else:
            cand = (oracle.primary_bucket(k, t.num_buckets), oracle.p2_alternate(k, t.num_buckets))
        assert all(occ[b] == t.bucket_slots for b in cand), (k, [occ[b] for b in cand])
