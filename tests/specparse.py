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


def _diff(c: int, r: int, op: int) -> int:
    """The difference operator: XOR (op 0), or each byte of c minus the byte
    of r modulo 256 (op 1)."""
    if op == 0:
        return c ^ r
    cb, rb = c.to_bytes(8, "little"), r.to_bytes(8, "little")
    return int.from_bytes(bytes((x - y) & 0xFF for x, y in zip(cb, rb)), "little")


def _bits_of(values, width):
    """Little-endian packing of a list of `width`-bit fields into bytes."""
    acc = 0
    for k, v in enumerate(values):
        acc |= v << (width * k)
    return acc.to_bytes((width * len(values) + 7) // 8, "little")


def _pad8(b: bytes) -> bytes:
    return b + b"\0" * (-len(b) % 8)


def encode_tad1(cur_records, ref_records, op: int = 0) -> bytes:
    """A plain-mode TAD1 encoding of current records against reference records
    (both lists of word lists), built bit by bit from the format's definition:
    a reference slot is matched by the current record with the same uid and
    header word; the residual runs over the matched records in reference
    order; per 64-word group the packer keeps one 4-bit length per non-zero
    word (the number of bytes up to and including its highest non-zero byte,
    found here from the bit length) and those low bytes."""
    by_key = {}
    for i, c in enumerate(cur_records):
        by_key[(c[0], c[1])] = i
    partner = [by_key.get((r[0], r[1]), -1) for r in ref_records]
    used = {i for i in partner if i >= 0}
    new = [i for i in range(len(cur_records)) if i not in used]
    D = []
    for j, r in enumerate(ref_records):
        if partner[j] >= 0:
            D += [_diff(c, x, op) for c, x in zip(cur_records[partner[j]], r)]
    W = len(D)
    G = (W + 63) // 64
    presence = _bits_of([1 if p >= 0 else 0 for p in partner], 1)
    presence += b"\0" * (8 * ((len(ref_records) + 63) // 64) - len(presence))
    word_bits = b""
    sizes = []
    blocks = b""
    for g in range(G):
        words = D[64 * g: 64 * g + 64]
        word_bits += _bits_of([1 if w else 0 for w in words] + [0] * (64 - len(words)), 1)
        nz = [w for w in words if w]
        lens = [(w.bit_length() + 7) // 8 for w in nz]
        nibbles = _bits_of(lens, 4)
        sig = b"".join(w.to_bytes(8, "little")[:n] for w, n in zip(nz, lens))
        blk = _pad8(nibbles + sig)
        sizes.append(len(blk) // 8)
        blocks += blk
    new_sizes = [len(cur_records[i]) for i in new]
    new_words = sum(new_sizes)
    fold = 0
    for r in ref_records:
        fold ^= r[0]
    hdr = struct.pack("<IHBBIIIIQQQQQ", int.from_bytes(b"TAD1", "little"), 1, 0, 1, len(ref_records),
                      len(ref_records) - partner.count(-1), len(new), op, sum(len(r) for r in ref_records), fold,
                      W, new_words, len(blocks))
    body = presence + word_bits + _pad8(bytes(sizes)) + _pad8(struct.pack(f"<{len(new)}I", *new_sizes))
    body += b"".join(struct.pack(f"<{len(cur_records[i])}Q", *cur_records[i]) for i in new)
    return hdr + body + blocks


def group_blocks(enc: bytes):
    """The residual groups of one TAD1 encoding: (mode, [(size byte, bitmap
    word, block bytes), ...]) in group order."""
    (magic, ver, mode, packer, n_ref, n_match, n_new, op, ref_words, fold, W, new_words,
     var_bytes) = struct.unpack_from("<IHBBIIIIQQQQQ", enc, 0)
    at = 64 + 8 * ((n_ref + 63) // 64)
    G = (W + 63) // 64
    bits = [struct.unpack_from("<Q", enc, at + 8 * g)[0] for g in range(G)]
    at += 8 * G
    gsz = list(enc[at:at + G])
    at += (G + 7) // 8 * 8
    at += (4 * n_new + 7) // 8 * 8 + 8 * new_words
    out = []
    for g in range(G):
        n = 8 * (gsz[g] & 0x7F)
        out.append((gsz[g], bits[g], bytes(enc[at:at + n])))
        at += n
    return mode, out
