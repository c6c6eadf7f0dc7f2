"""CPU interpreter of the packed instance table (host-logic tests only).

It evaluates, for every kernel vector x of a small instance, the same
predicate the GPU sweep evaluates from the table: the bit-sliced ridge slots
(at least 3 of a ridge's slot bits set = the ridge has degree 4), the facet
count bound and x != 0.  It also replays the kernel's walk over Gray
blocks (incremental fast-filter state; each candidate's full state rebuilt
from the item's reference state, lane tables, segment rows and the Gray-bit
tables) so the walk's bookkeeping is checked without a GPU.
"""
import numpy as np

HDR = 16


def header(tab):
    h = [int(v) for v in tab[:HDR]]
    return dict(k=h[1], kp=h[2], M=h[3], W=h[4], G=h[5], QS=h[6], RS=h[7], maxf=h[8],
                offset=bool(h[11] & 1), props_at=h[12], nprops=h[13], defer_at=h[14], ndefer=h[15])


def deferred(tab):
    """Parent facet indices of each deferred ridge."""
    h = header(tab)
    out, at = [], h["defer_at"]
    for _ in range(h["ndefer"]):
        p = int(tab[at])
        out.append([int(v) for v in tab[at + 1:at + 1 + p]])
        at += 1 + p
    return out


def offset_row(tab):
    """The coset offset K* in row layout (zeros for a linear span)."""
    h = header(tab)
    if not h["offset"]:
        return np.zeros(h["RS"], dtype=np.uint64)
    at = HDR + h["kp"] * h["RS"]
    return tab[at:at + h["RS"]].astype(np.uint64)


def properties(tab):
    """[(c0, [(weight, mask words)...])...] from the property section."""
    h = header(tab)
    out, at = [], h["props_at"]
    for _ in range(h["nprops"]):
        c0 = int(np.int32(np.uint32(tab[at])))
        ncls = int(tab[at + 1])
        at += 2
        cls = []
        for _ in range(ncls):
            cls.append((int(np.int32(np.uint32(tab[at]))), [int(v) for v in tab[at + 1:at + 1 + h["W"]]]))
            at += 1 + h["W"]
        out.append((c0, cls))
    return out


def rows(tab):
    h = header(tab)
    return tab[HDR:HDR + h["kp"] * h["RS"]].reshape(h["kp"], h["RS"]).astype(np.uint64)


def at_least3(words):
    c1 = np.zeros_like(words[0]); c2 = np.zeros_like(words[0]); c3 = np.zeros_like(words[0])
    for w in words:
        c3 |= c2 & w
        c2 |= c1 & w
        c1 |= w
    return c3


def state(R, x):
    v = np.zeros(R.shape[1], dtype=np.uint64)
    t = 0
    while x:
        if x & 1:
            v ^= R[t]
        x >>= 1
        t += 1
    return v


def slots4(v, base):
    """4-word groups are stored as (a, a^b, c, c^d)."""
    a, u, c, w = v[base], v[base + 1], v[base + 2], v[base + 3]
    return [a, a ^ u, c, c ^ w]


def accept(h, v):
    if at_least3(slots4(v, 0)) != 0:
        return False
    for g in range(1, h["G"]):
        base = 4 + (g - 1) * h["QS"]
        words = slots4(v, base) if h["QS"] == 4 else [v[base + q] for q in range(h["QS"])]
        if at_least3(words) != 0:
            return False
    koff = 4 + (h["G"] - 1) * h["QS"]
    cnt = sum(bin(int(v[koff + w])).count("1") for w in range(h["W"]))
    if not (h["maxf"] == 0 or cnt <= h["maxf"]):
        return False
    for parents in h.get("deferred", []):
        if sum((int(v[koff + f // 32]) >> (f % 32)) & 1 for f in parents) > 2:
            return False
    for c0, cls in h.get("props", []):
        g = c0
        for wgt, mask in cls:
            g += wgt * sum(bin(int(v[koff + w]) & mask[w]).count("1") for w in range(h["W"]))
        if g <= 0:
            return False
    return True


def survivors_direct(tab):
    h = header(tab)
    h["props"] = properties(tab)
    h["deferred"] = deferred(tab)
    R = rows(tab)
    off = offset_row(tab)
    first = 0 if h["offset"] else 1    # x = 0 is K* in a coset, else the empty complex
    return sorted(x for x in range(first, 1 << h["k"]) if accept(h, state(R, x) ^ off))


LANE_BITS = 9  # an item's lane chunks lie in one aligned window of 2^9 chunks


def _xor_rows(R, kp, first_row, v, nbits):
    """XOR of the rows first_row + j over the set bits j < nbits of v (rows
    >= kp count as zero)."""
    out = np.zeros(R.shape[1], dtype=np.uint64)
    for j in range(nbits):
        if (v >> j) & 1 and first_row + j < kp:
            out ^= R[first_row + j]
    return out


def survivors_walk(tab, cbits=7, lanes=64, offset_first=0):
    """Replays the GPU walk: items of `lanes` consecutive chunks of 2^cbits
    Gray indices, the item's first chunk a multiple of `lanes` (plus
    offset_first, to exercise unaligned windows).

    The fast filter follows the 4 group-0 words step by step.  A passing step
    r of segment sg of lane l is rebuilt from tables alone, as the kernel's
    check does: x = gray(i) for i = ((ref + d) << c) + (sg << 12) + r, with
    ref the item's first chunk rounded down to a multiple of 2^LANE_BITS and
    d = the lane's offset from it; by linearity of the Gray code its state is
      Ref                 rows of gray(ref << c) (the offset row included)
      ^ Lane(d)           rows c - 1 + i over the bits i of d ^ (d << 1),
                          from four tables of bits 0-2, 3-5, 6-8, 9
      ^ Seg(sg)           rows 12 + j over the bits j of gray(sg)
      ^ S(g12)            rows of the Gray bits 0-11 of r, bit 11 toggled by
                          the segment parity, from four tables of 3 bits.
    Every rebuilt state is compared with the direct sum of the rows of x.
    """
    h = header(tab)
    R = rows(tab)
    off = offset_row(tab)
    h["props"] = properties(tab)
    h["deferred"] = deferred(tab)
    kp, k = h["kp"], h["k"]
    c = min(max(cbits, 7), kp)
    T = np.zeros((4, 8, R.shape[1]), dtype=np.uint64)
    for b in range(4):
        for v in range(8):
            T[b][v] = _xor_rows(R, kp, 3 * b, v, 3)
    chunks = 1 << (kp - c)
    out = []
    first = 0
    items = []
    while first < chunks:
        f = min(chunks, first + offset_first) if first == 0 and offset_first else first
        n = min(lanes, chunks - f)
        if first == 0 and offset_first:
            items.append((0, min(chunks, offset_first)))
        items.append((f, n))
        first = f + n
    for first, n in items:
        if n <= 0:
            continue
        ref = first & ~((1 << LANE_BITS) - 1)
        assert (first - ref) + n <= (1 << LANE_BITS), "lane window crosses an aligned group"
        iref = ref << c
        xref = iref ^ (iref >> 1)
        Ref = off.copy()
        for t in range(kp):
            if (xref >> t) & 1:
                Ref ^= R[t]
        L = [[_xor_rows(R, kp, c - 1 + 3 * b, v, 3 if b < 3 else 1) for v in range(8)] for b in range(4)]
        for l in range(n):
            d = (first - ref) + l
            g = d ^ (d << 1)
            lane = Ref ^ L[0][g & 7] ^ L[1][(g >> 3) & 7] ^ L[2][(g >> 6) & 7] ^ L[3][(g >> 9) & 1]
            i0 = (first + l) << c
            s4 = lane[:4].copy()
            seg_row = np.zeros(R.shape[1], dtype=np.uint64)
            nblk = 1 << (c - 6)
            for blk in range(nblk):
                cand = []
                for s in range(64):
                    if at_least3(slots4(s4, 0)) == 0:
                        cand.append(s)
                    if s < 63:
                        t = (s + 1 & -(s + 1)).bit_length() - 1
                        s4 ^= R[t, :4]
                seg = blk >> 6
                for s in cand:
                    r12 = ((blk & 63) << 6) | s
                    g12 = (r12 ^ (r12 >> 1)) ^ ((seg & 1) << 11)
                    v = (lane ^ seg_row ^ T[0][g12 & 7] ^ T[1][(g12 >> 3) & 7] ^ T[2][(g12 >> 6) & 7]
                         ^ T[3][g12 >> 9])
                    i = i0 + (seg << 12) + r12
                    x = i ^ (i >> 1)
                    assert np.array_equal(v, state(R, x) ^ off), (first, l, blk, s)
                    if (x or h["offset"]) and (x >> k) == 0 and accept(h, v):
                        out.append(x)
                if blk + 1 < nblk:
                    t = 6 + ((blk + 1) & -(blk + 1)).bit_length() - 1
                    if t >= 12:
                        seg_row ^= R[t]
                    s4 ^= R[t, :4]
    return sorted(out)


def facets_of_x(basis, facets, x, offset=None):
    W = basis.shape[1] if basis.ndim == 2 and basis.shape[0] else (len(facets) + 31) // 32
    K = np.zeros(W, dtype=np.uint32) if offset is None else np.array(offset, dtype=np.uint32)
    t = 0
    while x:
        if x & 1:
            K ^= basis[t]
        x >>= 1
        t += 1
    return tuple(sorted(int(facets[w * 32 + b]) for w in range(W) for b in range(32)
                        if (int(K[w]) >> b) & 1))
