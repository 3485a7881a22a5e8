"""Host model of the LDS layouts that the BF16 backward kernels read with gfx950's transposing
read (ds_read_b64_tr_b16).  The address formulas of the kernels are restated here and checked
for (1) the transpose identity: a tile staged from its row-major MFMA operands and read back
with the transposing read gives the feature-major operand in the row order the products
expect, and (2) no LDS bank conflicts inside one access phase (64 banks of 4 bytes; 8 lanes
per phase of a 16-byte access, 16 lanes per phase of an 8-byte access).

Lane mapping of the transposing read, as measured on the device with an in-bounds probe: in
each group of 16 lanes, lane 4t + u supplies the address of 4 consecutive 16-bit values and
lane 4u + c receives value c of lane 4t + u as its value t."""
import itertools

BANKS = 64


def tile_idx(r, h):
    return 8 * (r >> 2) + 4 * h + (r & 3)


def tr_read(addr_of_lane, mem):
    """The transposing read: addr_of_lane(lane) -> element address; returns out[lane] = 4 values."""
    out = {}
    for g in range(4):
        for i in range(16):
            u, c = i >> 2, i & 3
            out[16 * g + i] = [mem[addr_of_lane(16 * g + 4 * t + u) + c] for t in range(4)]
    return out


def conflict_free(addrs_bytes, width):
    """One access phase: every lane's `width` bytes on banks no other lane of the phase uses."""
    used = set()
    for a in addrs_bytes:
        for b in range(a // 4, (a + width) // 4):
            if b % BANKS in used:
                return False
            used.add(b % BANKS)
    return True


# ---------------------------------------------------------------- attention backward (n <= 32)
def rsw(u, row):
    return (u & 4) | ((u & 3) ^ ((((row >> 1) & 1) << 1) | ((row >> 2) & 1)))


def stage_r_addr(fb, s, lr, h):
    """Element address of the 16-byte write of operand s by lane (lr, h), feature block fb."""
    return lr * 64 + rsw(4 * fb + 2 * s + h, lr) * 8


def tr_off(row, lane):
    g, u = lane >> 4, lane & 3
    return row * 64 + rsw(2 * (g & 1) + (u & 1), row) * 8 + 4 * (u >> 1)


def toff(lane):
    h = lane >> 5
    return tr_off(4 * h + ((lane & 15) >> 2), lane)


def test_attention_staging_transposes():
    for fb in range(2):
        mem = {}
        for lr, h, s in itertools.product(range(32), range(2), range(2)):
            base = stage_r_addr(fb, s, lr, h)
            for t in range(8):  # operand s, value t: feature 32 fb + tile_idx(8 s + t, h) of row lr
                mem[base + t] = (lr, 32 * fb + tile_idx(8 * s + t, h))
        assert len(mem) == 32 * 32
        for s in range(2):
            got = {}
            for rd in range(2):
                off = lambda lane, rd=rd: toff(lane) + (16 * s + 8 * rd) * 64 + 32 * fb
                for lane, vals in tr_read(off, mem).items():
                    got.setdefault(lane, []).extend(vals)
            for lane, vals in got.items():
                h = lane >> 5
                assert vals == [(tile_idx(8 * s + t, h), 32 * fb + lane % 32) for t in range(8)]


def test_attention_staging_conflict_free():
    for fb, s in itertools.product(range(2), range(2)):
        lanes = [(lane & 31, lane >> 5) for lane in range(64)]
        for p in range(8):  # 16-byte writes: 8 lanes per phase
            assert conflict_free([2 * stage_r_addr(fb, s, lr, h) for lr, h in lanes[8 * p: 8 * p + 8]], 16)
    for s, rd, fb in itertools.product(range(2), range(2), range(2)):
        for g in range(4):  # 8-byte transposing reads: 16 lanes per phase
            addrs = [2 * (toff(lane) + (16 * s + 8 * rd) * 64 + 32 * fb) for lane in range(16 * g, 16 * g + 16)]
            assert conflict_free(addrs, 8)


def test_attention_staging_halves_disjoint():
    # the two waves of a block stage feature blocks 0 and 1 of the same matrix: disjoint elements
    a = {stage_r_addr(0, s, lr, h) + t for s, lr, h, t in itertools.product(range(2), range(32), range(2), range(8))}
    b = {stage_r_addr(1, s, lr, h) + t for s, lr, h, t in itertools.product(range(2), range(32), range(2), range(8))}
    assert not a & b and len(a) == len(b) == 1024 and max(a | b) < 32 * 64


# ---------------------------------------------------------------- feed-forward backward (8 waves)
XS = 72  # row stride of the 64-wide tiles


def mlp_toff(lane):
    h = lane >> 5
    return (4 * h + ((lane & 15) >> 2)) * XS + 16 * ((lane >> 4) & 1) + 8 * (lane & 1) + 4 * ((lane >> 1) & 1)


def test_mlp_tiles_transpose():
    # x staged row-major: row r, position 32 sob + 16 s + 8 h + t holds feature 32 sob + tile_idx(8 s + t, h)
    mem = {}
    for r, sob, s, h, t in itertools.product(range(64), range(2), range(2), range(2), range(8)):
        mem[r * XS + 32 * sob + 16 * s + 8 * h + t] = (r, 32 * sob + tile_idx(8 * s + t, h))
    for rb, s, i in itertools.product(range(2), range(2), range(2)):
        got = {}
        for rd in range(2):
            off = lambda lane, rd=rd: mlp_toff(lane) + (32 * rb + 16 * s) * XS + 32 * i + 8 * rd * XS
            for lane, vals in tr_read(off, mem).items():
                got.setdefault(lane, []).extend(vals)
        for lane, vals in got.items():
            h = lane >> 5
            assert vals == [(32 * rb + tile_idx(8 * s + t, h), 32 * i + lane % 32) for t in range(8)]


def test_mlp_tiles_conflict_free():
    for base in (0, 16 * XS, 32 * XS + 32):
        for rd in range(2):
            for g in range(4):
                addrs = [2 * (mlp_toff(lane) + base + 8 * rd * XS) for lane in range(16 * g, 16 * g + 16)]
                assert conflict_free(addrs, 8)
    # du written as (hidden x row): lane (hidden 32 w + lr, h) writes 16 bytes at row position 32 rb + 16 s + 8 h
    for rb, s in itertools.product(range(2), range(2)):
        lanes = [(lane & 31, lane >> 5) for lane in range(64)]
        for p in range(8):
            assert conflict_free([2 * (lr * XS + 32 * rb + 16 * s + 8 * h) for lr, h in lanes[8 * p: 8 * p + 8]], 16)
