"""Host emulation of the one-workgroup solve's records (helper of
tests/test_local_layout.py; not a test module).

It runs the records exactly as the two waves of the kernel read them: an LDS
image of 8-byte slots, records copied into the FIFO at their offsets, fills
from b or from the x that has been drained so far, the groups of four
entries per lane (a row header sets acc = b_i and takes the diagonal, every
other entry subtracts its product, the division of Eq. (2.1) is stored at
ring slot (g mod 128) * 64 + lane where a row ends), drains to x.

The helper is played adversarially: it copies records as far ahead as their
FIFO waits allow and drains only when something needs it.  Then any wrong
wait or overlap in the layout reads a value that is not there yet (x starts
as NaN) or one that was overwritten, and the result differs from the
oracle's.  Every IEEE operation is a separate numpy operation in binary64,
so no fused multiply-add enters.
"""
from __future__ import annotations

import numpy as np

RING_GROUPS = 128
RING = RING_GROUPS * 64
ZERO = RING
FIFO0 = RING + 64                 # first FIFO slot (a block after the zero slot)
FIFO_BYTES = 189 * 512
SLOTS = FIFO0 + FIFO_BYTES // 8
GROUP = 2560
HDR = 32


class DeadlockError(AssertionError):
    pass


def run(rec: np.ndarray, info: np.ndarray, b: np.ndarray, n: int, lazy_drain: bool = True) -> np.ndarray:
    rec = np.ascontiguousarray(rec, dtype=np.uint8)
    info = np.ascontiguousarray(info, dtype=np.uint32).reshape(-1, 4)
    nrec = info.shape[0]
    lds = bytearray(SLOTS * 8)
    f64 = np.frombuffer(lds, dtype=np.float64)
    f64[:FIFO0] = np.nan
    f64[ZERO] = 0.0
    fifo_base = FIFO0 * 8
    x = np.full(n, np.nan)
    src_off = np.concatenate([[0], np.cumsum(info[:, 0].astype(np.int64))])

    st = {"staged": 0, "computed": 0, "drained": 0}
    offs = {}

    def hdr(r):
        o = fifo_base + offs[r]
        return np.frombuffer(lds, dtype=np.uint32, count=8, offset=o)

    def drain_to(target):
        if target > st["computed"]:
            raise DeadlockError(f"drain to {target} with only {st['computed']} computed")
        for r in range(st["drained"], target):
            h = hdr(r)
            ng, nf, nd = int(h[0]), int(h[1]), int(h[2])
            o = fifo_base + offs[r] + HDR + ng * GROUP + nf * 8
            d = np.frombuffer(lds, dtype=np.uint32, count=2 * nd, offset=o).reshape(-1, 2)
            x[d[:, 1].astype(np.int64)] = f64[d[:, 0].astype(np.int64)]
        st["drained"] = max(st["drained"], target)

    def stage_more():
        while st["staged"] < nrec:
            r = st["staged"]
            nbytes, foff, wait = int(info[r, 0]), int(info[r, 1]), int(info[r, 2])
            if wait > st["computed"]:
                return
            # the records whose bytes this copy reuses must be drained first
            drain_to(max(st["drained"], wait))
            lds[fifo_base + foff:fifo_base + foff + nbytes] = rec[src_off[r]:src_off[r] + nbytes].tobytes()
            offs[r] = foff
            h = hdr(r)
            ng, nf, need_far = int(h[0]), int(h[1]), int(h[5])
            if need_far > st["drained"]:
                if need_far > st["computed"]:
                    return      # the kernel's helper waits here too
                drain_to(need_far)
            o = fifo_base + foff + HDR + ng * GROUP
            fl = np.frombuffer(lds, dtype=np.uint32, count=2 * nf, offset=o).reshape(-1, 2)
            slot = (fl[:, 0] & 0x7FFFFFFF).astype(np.int64)
            # the kernel writes fill i to the i-th slot of the whole blocks after
            # the copied bytes, whatever the entry says: the two must agree
            slot0 = FIFO0 + (foff + (nbytes + 511) // 512 * 512) // 8
            assert np.array_equal(slot, slot0 + np.arange(nf)), ("fill slots", r)
            assert slot0 % 64 == 0 and foff % 512 == 0
            from_x = (fl[:, 0] & 0x80000000) != 0
            row = fl[:, 1].astype(np.int64)
            f64[slot] = np.where(from_x, x[row], b[row])
            st["staged"] = r + 1

    acc = np.zeros(64)
    diag = np.ones(64)
    lanes = np.arange(64)
    ring = 0
    off = 0
    with np.errstate(all="ignore"):
        for t in range(nrec):
            stage_more()
            if st["staged"] <= t:
                raise DeadlockError(f"record {t} never staged")
            h = hdr(t)
            ng, need_drain, nxt = int(h[0]), int(h[3]), int(h[4])
            assert offs[t] == off, (t, offs[t], off)
            if need_drain > st["drained"]:
                drain_to(need_drain)
            g0 = fifo_base + off + HDR
            for i in range(ng):
                gp = g0 + i * GROUP
                v = np.frombuffer(lds, dtype=np.float64, count=256, offset=gp).reshape(2, 64, 2)
                o = np.frombuffer(lds, dtype=np.uint16, count=256, offset=gp + 2048).reshape(64, 4).astype(np.int64)
                start = (o[:, 0] & 0x8000) != 0
                end = (o[:, 1] & 0x8000) != 0
                x0 = f64[o[:, 0] & 0x7FFF]
                x1 = f64[o[:, 1] & 0x7FFF]
                x2 = f64[o[:, 2]]
                x3 = f64[o[:, 3]]
                a = np.where(start, x0, acc - v[0, :, 0] * x0)
                diag = np.where(start, v[0, :, 0], diag)
                a = a - v[0, :, 1] * x1
                a = a - v[1, :, 0] * x2
                a = a - v[1, :, 1] * x3
                acc = a
                if end.any():
                    f64[ring * 64 + lanes] = a / diag
                ring = (ring + 1) % RING_GROUPS
            st["computed"] = t + 1
            off = nxt
            if not lazy_drain:
                drain_to(st["computed"])
        drain_to(nrec)
    return x
