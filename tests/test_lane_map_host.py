"""Host check (no GPU) of the property the one-launch chunk starts rely on.

Wave task v walks the chunks c = 2 (64 (v >> 1) + lane) + (v & 1), lane = 0..63,
and a chunk of 2^b terms starts at Gray index c 2^b, code gray(c 2^b) (App. A).
The 64 start codes of a wave agree in every bit outside b..b+6, so the part of
the start row sums from those columns is one vector per wave; bits b..b+6 each
take both values among the lanes, so no smaller set of columns would do.
"""


def gray(k):
    return k ^ (k >> 1)


def chunk(v, lane):
    return 2 * (64 * (v >> 1) + lane) + (v & 1)


def test_lanes_share_all_gray_bits_outside_b_to_b_plus_6():
    for b in range(1, 25):
        own = 0x7F << b
        for v in (0, 1, 2, 3, 6, 7, 1000, 1001, 2 ** 20 + 5):
            codes = [gray(chunk(v, lane) << b) for lane in range(64)]
            first = codes[0]
            assert all((x ^ first) & ~own == 0 for x in codes), (b, v)
            varying = 0
            for x in codes:
                varying |= x ^ first
            assert varying == own, (b, v, hex(varying))


def test_each_chunk_once():
    seen = set()
    for v in range(256):
        for lane in range(64):
            seen.add(chunk(v, lane))
    assert seen == set(range(256 * 64))
