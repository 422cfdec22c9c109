"""Brute-force twin of the oracle map -- TEST INFRASTRUCTURE ONLY.

A list of (key, value) pairs searched by linear scan, in pure Python, for tiny
inputs.  It restates the paper's API (Section 5.1: Upsert with a callback,
Query, Erase; insert = upsert with the "insert if unique" callback) without
sharing anything with `hw_oracle.cpp` beyond the meaning of the status codes, so
that the two agreeing on random batches pins the C++ map.
"""


def brute_apply(pairs, ops, keys, vals, combine, key_bits=64, capacity=0):
    """Apply ops in order to `pairs` (a list of [key, value] lists, mutated).

    ops: 0 query, 1 insert, 2 upsert, 3 erase.  combine: 0 sum, 1 keep, 2 replace,
    3 min, 4 max.  Returns (status list, value-out list)."""
    mask = (1 << key_bits) - 1
    reserved = 3 if key_bits == 64 else 2
    status, outs = [], []
    for i, op in enumerate(ops):
        k = int(keys[i])
        v = int(vals[i]) & mask if vals is not None else 0
        # linear scan for the key
        where = -1
        for idx in range(len(pairs)):
            if pairs[idx][0] == k:
                where = idx
                break
        st, out = 0, 0
        if k > mask - reserved:
            st = 4
        elif op == 0:
            if where >= 0:
                st, out = 1, pairs[where][1]
        elif op in (1, 2):
            c = 1 if op == 1 else combine
            if where >= 0:
                old = pairs[where][1]
                if c == 0:
                    new = (old + v) % (mask + 1)
                elif c == 1:
                    new = old
                elif c == 2:
                    new = v
                elif c == 3:
                    new = v if v < old else old
                else:
                    new = v if v > old else old
                pairs[where][1] = new
                st = 2
            elif capacity and len(pairs) >= capacity:
                st = 3
            else:
                pairs.append([k, v])
                st = 1
        elif op == 3:
            if where >= 0:
                pairs.pop(where)
                st = 1
        else:
            raise ValueError(op)
        status.append(st)
        outs.append(out)
    return status, outs
