"""Independent readers of the wire formats, written from their definition,
used to pin the oracle: a TAM1 message parser and a TAD1 decoder in plain
Python (no shared code with either implementation)."""
import struct


def parse_tam1(buf: bytes):
    """-> list of records, each a list of 8-byte little-endian words (ints)."""
    magic, ver, flags, n, pad, rec_words, reserved = struct.unpack_from("<IHHIIQQ", buf, 0)
    assert magic == int.from_bytes(b"TAM1", "little") and ver == 1 and flags == 0 and pad == 0 and reserved == 0
    offs = list(struct.unpack_from(f"<{n}I", buf, 32))
    table = 8 * ((n + 1) // 2)
    if n % 2:
        assert struct.unpack_from("<I", buf, 32 + 4 * n)[0] == 0
    area = 32 + table
    assert len(buf) == area + 8 * rec_words
    recs = []
    for i in range(n):
        at = area + 8 * offs[i]
        words = struct.unpack_from("<Q", buf, at + 8)[0] >> 32
        recs.append(list(struct.unpack_from(f"<{words}Q", buf, at)))
    return recs


def _undiff(r: int, d: int, op: int) -> int:
    """Invert the difference operator: XOR (op 0), or add each byte of d to
    the byte of r modulo 256 (op 1)."""
    if op == 0:
        return r ^ d
    rb, db = r.to_bytes(8, "little"), d.to_bytes(8, "little")
    return int.from_bytes(bytes((x + y) & 0xFF for x, y in zip(rb, db)), "little")


def decode_tad1(enc: bytes, ref_records):
    """Decode a plain-mode TAD1 against the reference records -> records of C'."""
    (magic, ver, mode, packer, n_ref, n_match, n_new, op, ref_words, fold, W, new_words,
     var_bytes) = struct.unpack_from("<IHBBIIIIQQQQQ", enc, 0)
    assert magic == int.from_bytes(b"TAD1", "little") and ver == 1 and packer == 1 and mode == 0
    assert op in (0, 1)
    assert n_ref == len(ref_records)
    at = 64
    pres = int.from_bytes(enc[at:at + 8 * ((n_ref + 63) // 64)], "little")
    at += 8 * ((n_ref + 63) // 64)
    G = (W + 63) // 64
    bits = int.from_bytes(enc[at:at + 8 * G], "little")
    at += 8 * G
    gsz = list(enc[at:at + G])
    at += (G + 7) // 8 * 8
    sizes = list(struct.unpack_from(f"<{n_new}I", enc, at))
    at += (4 * n_new + 7) // 8 * 8
    new_area = at
    at += 8 * new_words
    # residual words
    D = [0] * W
    for g in range(G):
        blk = enc[at:at + 8 * gsz[g]]
        nz = [q for q in range(64 * g, min(W, 64 * g + 64)) if (bits >> q) & 1]
        nib = [(blk[t // 2] >> (4 * (t % 2))) & 15 for t in range(len(nz))]
        p = (len(nz) + 1) // 2
        for q, ln in zip(nz, nib):
            D[q] = int.from_bytes(blk[p:p + ln], "little")
            p += ln
        at += 8 * gsz[g]
    assert at == len(enc)
    out, q = [], 0
    for j, rec in enumerate(ref_records):
        if (pres >> j) & 1:
            out.append([_undiff(a, b, op) for a, b in zip(rec, D[q:q + len(rec)])])
            q += len(rec)
    p = new_area
    for s in sizes:
        out.append(list(struct.unpack_from(f"<{s}Q", enc, p)))
        p += 8 * s
    return out
