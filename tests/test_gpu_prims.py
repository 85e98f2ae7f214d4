"""GPU checks of the build's two device-wide primitives against their plain
definitions: the stable LSD radix sort (order by the low `bits` bits, equal
keys keep their input order, the payload moves with its key) and the batched
exclusive prefix sums (out[i] = in[0] + ... + in[i-1], total = the sum).  The
sizes cross every tiling regime of the sort (1024-, 2048- and 4096-key tiles,
histogram workgroups over one and several groups of tiles) and both paths of
the batched scan (one launch pair, one scan at a time)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sba():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2010_12548_amd as m
    m.lib()
    return m


def keys_of(kind, n, rng):
    if kind == "random":
        return rng.integers(0, 2**63, n, dtype=np.int64) * 2 + rng.integers(0, 2, n)
    if kind == "equal":
        return np.full(n, 0x1234_5678_9abc_def0, dtype=np.int64)
    if kind == "sorted":
        return np.sort(rng.integers(0, 2**40, n, dtype=np.int64))
    if kind == "reverse":
        return np.sort(rng.integers(0, 2**40, n, dtype=np.int64))[::-1].copy()
    if kind == "few":
        return rng.integers(0, 5, n, dtype=np.int64) << 17
    raise ValueError(kind)


def check_sort(sba, keys, bits, with_vals=True):
    n = keys.shape[0]
    k = torch.from_numpy(keys).cuda()
    v = torch.arange(n, dtype=torch.int32, device="cuda") if with_vals else None
    sba.radix_sort(k, v, bits)
    torch.cuda.synchronize()
    mask = np.uint64((1 << bits) - 1) if bits < 64 else np.uint64(2**64 - 1)
    order = np.argsort(keys.view(np.uint64) & mask, kind="stable")
    np.testing.assert_array_equal(k.cpu().numpy(), keys[order])
    if with_vals:
        np.testing.assert_array_equal(v.cpu().numpy(), order.astype(np.int32))


@pytest.mark.parametrize("kind", ["random", "equal", "sorted", "reverse", "few"])
@pytest.mark.parametrize("n", [0, 1, 2, 1000, 1024 * 4 * 4 + 3, 262_145, 300_001, (2 << 20) + 1,
                               (4 << 20) + 17])
def test_radix_sort(sba, kind, n):
    rng = np.random.default_rng(n * 7 + len(kind))
    keys = keys_of(kind, n, rng)
    check_sort(sba, keys, 64 if kind == "random" else 48)


@pytest.mark.parametrize("bits", [1, 7, 8, 9, 17, 21, 26, 33, 35, 63, 64])
def test_radix_sort_bits(sba, bits):
    # keys below 2^bits, as every caller's are
    rng = np.random.default_rng(bits)
    keys = rng.integers(-2**63, 2**63 - 1, 200_003, dtype=np.int64)
    keys = (keys.view(np.uint64) & np.uint64(2**bits - 1)).view(np.int64)
    check_sort(sba, keys, bits)


@pytest.mark.parametrize("kind", ["random", "equal", "sorted", "reverse", "few"])
@pytest.mark.parametrize("n", [1000, 1024 * 4 * 4 + 3, 300_001])
def test_radix_sort_nine_bit_digits(sba, kind, n):
    # 35-bit keys (the build's event keys at city sizes) take four 9-bit
    # passes instead of five 8-bit ones
    rng = np.random.default_rng(n * 11 + len(kind))
    keys = keys_of(kind, n, rng)
    keys = (keys.view(np.uint64) & np.uint64(2**35 - 1)).view(np.int64)
    check_sort(sba, keys, 35)


@pytest.mark.parametrize("nbytes", [1, 3, 5, 7])
def test_radix_sort_ignores_bytes_above(sba, nbytes):
    # the passes cover whole bytes: bytes above them are not part of the
    # order, and equal low bytes keep their input order
    rng = np.random.default_rng(100 + nbytes)
    keys = rng.integers(-2**63, 2**63 - 1, 200_003, dtype=np.int64)
    check_sort(sba, keys, 8 * nbytes)


@pytest.mark.parametrize("n,bits", [(20_000_011, 40), (66_000_001, 24)])
def test_radix_sort_large(sba, n, bits):
    # 2048-key tiles with histogram workgroups over 3 groups of tiles, and
    # 4096-key tiles over 8 groups; the last workgroup holds a partial group
    rng = np.random.default_rng(n)
    keys = rng.integers(0, 2**62, n, dtype=np.int64)
    check_sort(sba, keys, bits, with_vals=n < 30_000_000)


def test_radix_sort_rejects(sba):
    k = torch.zeros(4, dtype=torch.int64, device="cuda")
    for bits in (0, 65):
        with pytest.raises(sba.SbaError):
            sba.radix_sort(k, None, bits)


SIZES = [0, 1, 2047, 2048, 2049, 100_000, 1 << 21, (1 << 21) + 1]


@pytest.mark.parametrize("in_place", [False, True])
@pytest.mark.parametrize("sizes", [
    [5, 0], [2048, 2049, 1], [100_000, 1, 0, 7777],          # one launch pair
    [1 << 21, 3, 1 << 21],                                    # at the limit
    [(1 << 21) + 1, 10],                                      # one by one (too long)
    [9, 8, 7, 6, 5],                                          # one by one (too many)
    [0, 0, 0],
])
def test_scan_multi(sba, sizes, in_place):
    rng = np.random.default_rng(sum(sizes) + len(sizes))
    host = [rng.integers(-10**6, 10**6, n, dtype=np.int64) for n in sizes]
    arrs = [torch.from_numpy(h).cuda() for h in host]
    outs, total = sba.scan_multi(arrs, in_place=in_place)
    torch.cuda.synchronize()
    tot = total.cpu().numpy()
    for k, h in enumerate(host):
        want = np.concatenate([[0], np.cumsum(h)[:-1]]) if h.size else h
        np.testing.assert_array_equal(outs[k].cpu().numpy(), want)
        assert tot[k] == h.sum()


def test_scan_multi_wide_values(sba):
    # tile sums far beyond 32 bits and of either sign (the build scans
    # packed counts): every bit of a tile sum must arrive
    rng = np.random.default_rng(5)
    sizes = [1 << 21, 300_001, 4097]
    host = [rng.integers(-2**40, 2**40, n, dtype=np.int64) for n in sizes]
    host[1] = np.abs(host[1]) << 2                       # sums near 2^60
    arrs = [torch.from_numpy(h).cuda() for h in host]
    outs, total = sba.scan_multi(arrs)
    torch.cuda.synchronize()
    tot = total.cpu().numpy()
    for k, h in enumerate(host):
        want = np.concatenate([[0], np.cumsum(h)[:-1]])
        np.testing.assert_array_equal(outs[k].cpu().numpy(), want)
        assert tot[k] == h.sum()


@pytest.mark.parametrize("nbytes", [0, 16, 4096 + 48, 64 * 1024 * 1024 + 16 * 7])
@pytest.mark.parametrize("blocks,threads", [(1, 64), (512, 512), (256, 1024)])
@pytest.mark.parametrize("two", [False, True])
def test_stream_read_reads_every_word(sba, nbytes, blocks, threads, two):
    # the streaming-read yardstick folds every 32-bit word of its buffers into
    # one XOR: any skipped or repeated 16-byte load changes it
    rng = np.random.default_rng(nbytes + blocks + 7 * two)
    words = rng.integers(0, 2**32, (2 if two else 1) * (nbytes // 4),
                         dtype=np.uint64).astype(np.uint32)
    data = torch.from_numpy(words.view(np.int32)).cuda()
    n = nbytes // 4
    if two:
        out = sba.stream_read(data[:n], data[n:], blocks=blocks, threads=threads)
    else:
        out = sba.stream_read(data, blocks=blocks, threads=threads)
    torch.cuda.synchronize()
    want = np.bitwise_xor.reduce(words) if words.size else np.uint32(0)
    assert np.uint32(out.cpu().numpy().view(np.uint32)[0]) == want


def test_stream_read_rejects(sba):
    data = torch.zeros(16, dtype=torch.int32, device="cuda")
    with pytest.raises(RuntimeError):
        sba.stream_read(data[1:5])                 # not 16-byte aligned
    with pytest.raises(RuntimeError):
        sba.stream_read(data[:6])                  # 24 bytes
    with pytest.raises(RuntimeError):
        sba.stream_read(data, blocks=0)
    with pytest.raises(RuntimeError):
        sba.stream_read(data, threads=96)
    with pytest.raises(ValueError):
        sba.stream_read(data[:8], data[:4])        # unequal sizes
