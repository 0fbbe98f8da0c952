"""Test-only numpy interpretation of a packed store (no GPU).

Reads the header and descriptor tables that hm_pack_host wrote and evaluates
the product the way the store's layout defines it (row panels, column tiles,
partial reduction for blocks over several column chunks, t straight from the
tiles for blocks inside one).  Used to check the block scheduler and the packer on the
CPU against the oracle; it shares no code with either.
"""

import numpy as np

HDR = np.dtype([("magic", "<u8"), ("n_rows", "<i8"), ("n_cols", "<i8"),
                ("n_row_panels", "<i8"), ("n_row_sections", "<i8"), ("n_col_tiles", "<i8"),
                ("n_tblocks", "<i8"), ("n_large", "<i8"), ("n_large_t", "<i8"), ("n_t", "<i8"),
                ("n_partials", "<i8"), ("off_row_panels", "<i8"), ("off_row_sections", "<i8"),
                ("off_row_order", "<i8"), ("off_row_src", "<i8"), ("off_col_tiles", "<i8"),
                ("off_col_dst", "<i8"), ("off_tblocks", "<i8"), ("off_large", "<i8"),
                ("off_owner", "<i8"), ("off_sigma", "<i8"), ("acc_dtype", "<i8"),
                ("has_sigma", "<i8"), ("off_p1_order", "<i8"), ("n_p1", "<i8"),
                ("off_p2_order", "<i8"), ("n_p2", "<i8"), ("n_red_t", "<i8"),
                ("has_aflp", "<i8"), ("off_row_aflp", "<i8"), ("off_col_aflp", "<i8")])
RP = np.dtype([("src_off", "<i8"), ("row0", "<i4"), ("m", "<i4"), ("ncols", "<i4"),
               ("sec0", "<i4"), ("nsec", "<i4"), ("pad", "<i4")])
RS = np.dtype([("data_off", "<i8"), ("dtype", "<i4"), ("ngroups", "<i4"), ("col0", "<i4"),
               ("pad", "<i4", (3,))])
CT = np.dtype([("data_off", "<i8"), ("nrows", "<i4"), ("x0", "<i4"), ("ngroups", "<i4"),
               ("dst_off", "<i4"), ("dtype", "u1", (4,)), ("end", "u1", (4,))])
TB = np.dtype([("pst", "<i4"), ("k", "<i4"), ("nseg", "<i4"), ("toff", "<i4")])
G = {0: 2, 1: 4, 2: 8, 3: 8, 4: 4, 5: 4, 6: 4, 7: 8, 8: 8, 9: 8, 10: 8, 11: 4, 12: 4, 13: 4, 14: 8, 15: 4, 16: 4}
# bytes per value inside the 16-byte groups
SZ = {0: 8, 1: 4, 2: 2, 3: 2, 4: 4, 5: 4, 6: 4, 7: 2, 8: 2, 9: 2, 10: 2, 11: 4, 12: 4, 13: 4, 14: 2, 15: 4, 16: 4}
# low bytes per value, bit position (DFL40 / 48 / 24, AFLP24 / 40 / 48)
LO = {5: (1, 24), 6: (2, 16), 8: (1, 40), 10: (1, 40), 12: (1, 24), 13: (2, 16), 14: (1, 40), 15: (1, 24),
      16: (2, 16)}
AFLP_BYTES = {9: 2, 10: 3, 11: 4, 12: 5, 13: 6}
BFL_BYTES = {14: 3, 15: 5, 16: 6}


def decode_bfl(code: np.ndarray, nbytes: int) -> np.ndarray:
    """BFL values from left-aligned 64-bit codes: sign, 8 exponent bits E
    (bias 127) and m = 8 nbytes - 9 fraction bits; 2^(E-127) (1 + f 2^-m),
    and zero for E = 0."""
    m = 8 * nbytes - 9
    c = code >> np.uint64(64 - 8 * nbytes)
    sign = np.where((c >> np.uint64(8 * nbytes - 1)) & np.uint64(1), -1.0, 1.0)
    E = ((c >> np.uint64(m)) & np.uint64(255)).astype(np.int64)
    f = (c & ((np.uint64(1) << np.uint64(m)) - np.uint64(1))).astype(np.float64)
    return np.where(E == 0, 0.0, sign * np.ldexp(1.0 + np.ldexp(f, -m), E - 127))


def decode_aflp(code: np.ndarray, prm: np.ndarray, nbytes: int) -> np.ndarray:
    """AFLP values from left-aligned 64-bit codes (uint64) and the int32
    parameter of each value's column (broadcast against code): k = prm >> 8,
    e = 11 - (prm & 255); the code is the sign, e bits of the binary
    exponent j of d and m = 8 nbytes - 1 - e bits of d's fraction; the value
    is sign (d - 1) 2^k with d = 2^j (1 + fraction 2^-m)."""
    prm = np.broadcast_to(prm, code.shape).astype(np.int64)
    k = prm >> 8
    e = 11 - (prm & 255)
    m = 8 * nbytes - 1 - e
    c = code >> np.uint64(64 - 8 * nbytes)                 # the nbytes-byte code
    sign = np.where((c >> np.uint64(8 * nbytes - 1)) & np.uint64(1), -1.0, 1.0)
    frac = (c & ((np.uint64(1) << m.astype(np.uint64)) - np.uint64(1))).astype(np.float64)
    j = ((c >> m.astype(np.uint64)) & ((np.uint64(1) << e.astype(np.uint64)) - np.uint64(1))).astype(np.int64)
    d = np.ldexp(1.0 + np.ldexp(frac, -m), j)
    return sign * np.ldexp(d - 1.0, k)


def dfl_code(hi: np.ndarray, lo, dt: int) -> np.ndarray:
    """Left-aligned 64-bit codes (uint64) from their leading words (uint32
    for the 4-byte-word formats, uint16 for the 2-byte ones) and, for the
    formats with a low-byte plane, their low bytes (uint8 / uint16 arrays of
    the same shape)."""
    bits = hi.astype(np.uint64) << np.uint64(64 - 8 * SZ[dt])
    if dt in LO:
        bits |= lo.astype(np.uint64) << np.uint64(LO[dt][1])
    return bits


def decode_dfl(hi: np.ndarray, lo, dt: int) -> np.ndarray:
    """DFL values: the codes are their FP64 encodings."""
    return dfl_code(hi, lo, dt).view("<f8")


def decode(buf: np.ndarray, off: int, count: int, dt: int) -> np.ndarray:
    raw = buf[off: off + count * SZ[dt]]
    if dt == 0:
        return raw.view("<f8").astype(np.float64)
    if dt == 1:
        return raw.view("<f4").astype(np.float64)
    if dt == 2:
        return raw.view("<f2").astype(np.float64)
    return (raw.view("<u2").astype(np.uint32) << 16).view("<f4").astype(np.float64)


def tables(buf: np.ndarray):
    h = buf[:HDR.itemsize].view(HDR)[0]
    def arr(dt, off, n):
        return buf[off: off + n * dt.itemsize].view(dt) if n else np.zeros(0, dt)
    return h, dict(
        row_aflp=buf[h["off_row_aflp"]:].view("<i4") if h["has_aflp"] else None,
        col_aflp=buf[h["off_col_aflp"]:].view("<i4") if h["has_aflp"] else None,
        rp=arr(RP, h["off_row_panels"], h["n_row_panels"]),
        rs=arr(RS, h["off_row_sections"], h["n_row_sections"]),
        order=arr(np.dtype("<i4"), h["off_row_order"], h["n_row_panels"]),
        ct=arr(CT, h["off_col_tiles"], h["n_col_tiles"]),
        tb=arr(TB, h["off_tblocks"], h["n_tblocks"]),
    )


def model_mvm(buf: np.ndarray, x: np.ndarray, y0: np.ndarray, alpha: float) -> np.ndarray:
    h, T = tables(buf)
    n_cols = int(h["n_cols"])
    part = np.zeros(int(h["n_partials"]))
    t_direct = np.zeros(int(h["n_t"]))
    written = np.zeros(int(h["n_t"]), bool)
    dst_all = buf[h["off_col_dst"]:].view("<i4")
    for t in T["ct"]:
        nr, ng = int(t["nrows"]), int(t["ngroups"])
        # a tile row is ng 16-byte groups, in runs of one format each
        d0 = int(t["data_off"])
        raw = buf[d0: d0 + nr * ng * 16].reshape(nr, ng * 16)
        # low-byte plane after the rows: one entry of Lt bytes per row and
        # group (the largest entry of the tile's formats)
        Lt = max(G[int(d)] * LO[int(d)][0] if int(d) in LO else 0 for d in t["dtype"])
        plane = buf[d0 + nr * ng * 16: d0 + nr * ng * (16 + Lt)].reshape(nr, ng, Lt) if Lt else None
        parts, g0 = [], 0
        parts_cols = []                                  # columns of the runs decoded so far
        for r in range(4):
            e, dt = int(t["end"][r]), int(t["dtype"][r])
            if e > g0:
                parts_cols.append(0)
                block = np.ascontiguousarray(raw[:, 16 * g0: 16 * e]).reshape(-1)
                if dt >= 4:
                    lo = None
                    if dt in LO:
                        nb = LO[dt][0]
                        lo = np.ascontiguousarray(plane[:, g0:e, : G[dt] * nb]).reshape(-1)
                        lo = lo.view("<u1" if nb == 1 else "<u2")
                    hi = block.view("<u4" if SZ[dt] == 4 else "<u2")
                    if dt in AFLP_BYTES:                 # parameters per tile column
                        c0 = int(t["dst_off"]) + sum(parts_cols)
                        prm = T["col_aflp"][c0: c0 + (e - g0) * G[dt]]
                        parts.append(decode_aflp(dfl_code(hi, lo, dt).reshape(nr, -1), prm[None, :],
                                                 AFLP_BYTES[dt]))
                    elif dt in BFL_BYTES:
                        parts.append(decode_bfl(dfl_code(hi, lo, dt), BFL_BYTES[dt]).reshape(nr, -1))
                    else:
                        parts.append(decode_dfl(hi, lo, dt).reshape(nr, -1))
                else:
                    parts.append(decode(block, 0, block.size // SZ[dt], dt).reshape(nr, -1))
                parts_cols[-1] = parts[-1].shape[1]
            g0 = e
        assert g0 == ng
        V = np.concatenate(parts, axis=1)                    # nr x cols (tile column order)
        cols = V.shape[1]
        p = V.T @ x[int(t["x0"]): int(t["x0"]) + nr]
        d = dst_all[int(t["dst_off"]): int(t["dst_off"]) + cols]
        part[d[d >= 0]] = p[d >= 0]
        direct = d <= -2                                     # t entry -d - 2 of a one-chunk block
        assert not np.any(written[-d[direct] - 2])
        t_direct[-d[direct] - 2] = p[direct]
        written[-d[direct] - 2] = True
    sig = None
    if h["has_sigma"]:
        sig = decode(buf, int(h["off_sigma"]), int(h["n_t"]), 0 if h["acc_dtype"] == 0 else 1)
    t_vec = np.zeros(int(h["n_t"]))
    n_red_t = int(h["n_red_t"])
    for b in T["tb"]:
        k, ns, pst, toff = int(b["k"]), int(b["nseg"]), int(b["pst"]), int(b["toff"])
        if ns == 1:                                          # from the column tiles
            assert toff >= n_red_t and pst == -1 and np.all(written[toff: toff + k])
            s = t_direct[toff: toff + k]
        else:
            assert toff + k <= n_red_t
            s = part[pst: pst + ns * k].reshape(ns, k).sum(0)
        t_vec[toff: toff + k] = s if sig is None else s * sig[toff: toff + k]
    z = np.concatenate([x, t_vec])
    src_all = buf[h["off_row_src"]:].view("<i4")
    y = np.array(y0, dtype=np.float64, copy=True)
    for p in T["rp"]:
        m = int(p["m"])
        src = src_all[int(p["src_off"]): int(p["src_off"]) + int(p["ncols"])]
        acc = np.zeros(m)
        for s in T["rs"][int(p["sec0"]): int(p["sec0"]) + int(p["nsec"])]:
            dt, ng, c0 = int(s["dtype"]), int(s["ngroups"]), int(s["col0"])
            g = G[dt]
            d0 = int(s["data_off"])
            if dt >= 4:
                hi = np.ascontiguousarray(buf[d0: d0 + ng * m * 16]).view("<u4" if SZ[dt] == 4 else "<u2")
                lo = None
                if dt in LO:                                 # low-byte plane after the groups
                    nb = LO[dt][0]
                    lo = np.ascontiguousarray(buf[d0 + ng * m * 16: d0 + ng * m * (16 + G[dt] * nb)])
                    lo = lo.view("<u1" if nb == 1 else "<u2")
                if dt in AFLP_BYTES:                         # parameters per source slot
                    s0 = int(p["src_off"]) + c0
                    prm = T["row_aflp"][s0: s0 + ng * g].reshape(ng, 1, g)
                    vals = decode_aflp(dfl_code(hi, lo, dt).reshape(ng, m, g), prm, AFLP_BYTES[dt])
                elif dt in BFL_BYTES:
                    vals = decode_bfl(dfl_code(hi, lo, dt), BFL_BYTES[dt]).reshape(ng, m, g)
                else:
                    vals = decode_dfl(hi, lo, dt).reshape(ng, m, g)
            else:
                vals = decode(buf, d0, ng * m * g, dt).reshape(ng, m, g)
            M = vals.transpose(1, 0, 2).reshape(m, ng * g)       # m x cols
            acc += M @ z[src[c0: c0 + ng * g]]
        y[int(p["row0"]): int(p["row0"]) + m] += alpha * acc
    return y
