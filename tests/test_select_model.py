"""A host model of the per-tile radix select (the most-significant-bit-first
walk over 32-bit score keys that the scoring kernels run on wavefront ballots)
against a brute-force sort, and of a variant that starts below the leading
bits every valid key shares (found from the largest and the smallest valid
key): both find the k-th largest key on random key sets with invalid (zero)
keys, ties, one sign only (the keys of non-negative scores all carry the top
bit) and mixed signs. Also the merge select's walk over 64-bit (score, id) keys in
12-bit digits, from the top bit and from below the prefix all keys share,
and the wide-k first pass's starting threshold taken from a share of each
sampled tile. Only the order-preserving key map of snn_device.h is shared with the library;
the walks are restated here."""
import numpy as np
import pytest


def ord_key(x):
    b = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    return np.where(b & 0x80000000, ~b & 0xFFFFFFFF, b | 0x80000000).astype(np.uint64)


def select_kth(keys, k, start_bit=31, prefix=0):
    """(threshold, exact, need) as the kernels return them: exact when the keys
    >= threshold number exactly k; otherwise the threshold is the k-th largest
    key and `need` keys equal to it are still to be taken."""
    need = k
    for bit in range(start_bit, -1, -1):
        hm = (0xFFFFFFFF << bit) & 0xFFFFFFFF
        want = prefix | (1 << bit)
        c = int(np.count_nonzero((keys & hm) == want))
        if c >= need:
            prefix = want
            if c == need:
                return prefix, True, 0
        else:
            need -= c
    return prefix, False, need


def select_kth_skip(keys, k):
    """The same walk started below the bits that the largest and the smallest
    valid (non-zero) key share; those bits are the prefix of every valid key."""
    valid = keys[keys != 0]
    mx, mn = int(valid.max()), int(valid.min())
    diff = mx ^ mn
    if diff == 0:
        return select_kth(keys, k)
    top = diff.bit_length() - 1  # highest bit where the valid keys differ
    prefix = mx & ~((1 << (top + 1)) - 1) & 0xFFFFFFFF
    return select_kth(keys, k, start_bit=top, prefix=prefix)


def brute(keys, k):
    s = np.sort(keys[keys != 0])[::-1]
    return int(s[k - 1]), int(np.count_nonzero(keys > s[k - 1]))


def check(keys, k):
    keys = keys.astype(np.uint64)
    kth, above = brute(keys, k)
    for T, exact, need in (select_kth(keys, k), select_kth_skip(keys, k)):
        if exact:
            assert np.count_nonzero(keys >= T) == k
            assert T <= kth and np.count_nonzero(keys >= T) == k
        else:
            assert T == kth and above == k - need and need >= 1
    a, b = select_kth(keys, k), select_kth_skip(keys, k)
    assert a == b, (a, b)


@pytest.mark.parametrize("law", ["exp", "normal", "ties", "narrow"])
def test_radix_select_model_against_a_sort(law):
    rng = np.random.default_rng({"exp": 1, "normal": 2, "ties": 3, "narrow": 4}[law])
    for trial in range(300):
        n = int(rng.integers(2, 1024))
        if law == "exp":
            s = rng.exponential(1.0, n)
        elif law == "normal":
            s = rng.standard_normal(n)
        elif law == "ties":
            s = rng.integers(0, 5, n).astype(np.float64)
        else:
            s = 1.0 + rng.integers(0, 64, n) * 2.0 ** -20  # keys equal in their top 20 bits
        keys = ord_key(s.astype(np.float32)).astype(np.uint64)
        keys[s == 0] = ord_key(np.float32(0.0))
        dead = rng.random(n) < rng.random() * 0.5  # slots not live or below the threshold
        keys[dead] = 0
        nv = int(np.count_nonzero(keys))
        if nv < 2:
            continue
        k = int(rng.integers(1, nv))  # the select runs when more than k keys are valid
        check(keys, k)


def digit_walk(keys, keep, start_at_prefix):
    """The merge select's walk over 64-bit keys, 12-bit digits at a time (a
    histogram of the next digit of the keys that share the prefix found so
    far, then the bin holding the need-th largest key), optionally started
    below the leading bits the largest and the smallest key share. Returns
    the threshold T: the result is every key >= T."""
    P, pb, need = 0, 0, keep
    if start_at_prefix:
        diff = int(keys.max()) ^ int(keys.min())
        if diff:
            pb = 64 - diff.bit_length()
            P = int(keys.max()) >> (64 - pb) if pb else 0
    while True:
        d = min(12, 64 - pb)
        sel = keys if pb == 0 else keys[(keys >> np.uint64(64 - pb)) == np.uint64(P)]
        digit = (sel >> np.uint64(64 - pb - d)) & np.uint64((1 << d) - 1)
        hist = np.bincount(digit.astype(np.int64), minlength=1 << d)
        above = 0
        for b in range((1 << d) - 1, -1, -1):
            if above < need <= above + hist[b]:
                break
            above += hist[b]
        in_bin, need = int(hist[b]), need - above
        P, pb = (P << d) | b, pb + d
        if in_bin == need or pb == 64:
            return P if pb == 64 else P << (64 - pb)


@pytest.mark.parametrize("law", ["exp", "narrow", "ties"])
def test_merge_select_digit_walk_against_a_sort(law):
    """The 64-bit digit walk of the merge select, from the top bit and from
    below the shared prefix, returns a threshold that exactly `keep` keys
    reach, the keep-th largest key, on distinct (score, id) keys whose scores
    share many leading bits (the candidates of a thresholded pass)."""
    rng = np.random.default_rng({"exp": 21, "narrow": 22, "ties": 23}[law])
    for trial in range(200):
        n = int(rng.integers(2, 3000))
        if law == "exp":
            s = 5.0 + rng.exponential(1.0, n)
        elif law == "narrow":
            s = 7.0 + rng.integers(0, 200, n) * 2.0 ** -18
        else:
            s = rng.integers(1, 4, n).astype(np.float64)
        ids = rng.choice(1 << 31, n, replace=False).astype(np.uint64)
        keys = (ord_key(s.astype(np.float32)) << np.uint64(32)) | (np.uint64(0xFFFFFFFF) - ids)
        keep = int(rng.integers(1, n)) if n > 1 else 1
        want = np.sort(keys)[::-1][keep - 1]
        for skip in (False, True):
            T = digit_walk(keys, keep, skip)
            assert np.count_nonzero(keys >= np.uint64(T)) == keep, (trial, skip)
            assert np.uint64(T) <= want


@pytest.mark.parametrize("seed", range(6))
def test_sampled_threshold_from_a_share_of_each_tile(seed):
    """The wide-k first pass lets each sampled tile keep only
    max(32, 4 k_s / tiles_s) of its best keys, and takes the lowest of the k_s
    best of what they keep as the starting threshold. What they keep is a
    subset of the sample, so that threshold is never above the sample's own
    k_s-th best (a lower threshold only lets more documents through); it equals
    it unless one tile held more of the k_s best than it kept, and with fewer
    than k_s kept in all there is no threshold. Checked on tiles of random
    scores, on tiles whose first few hold all the largest scores, and on tiles
    of few scores."""
    rng = np.random.default_rng(seed)
    tiles_s = int(rng.integers(4, 80))
    tile = 4096
    k = int(rng.integers(1000, 20001))
    tiles = tiles_s * 16
    k_s = (3 * k * tiles_s + 2 * tiles - 1) // (2 * tiles) + 32
    share = max(32, (4 * k_s + tiles_s - 1) // tiles_s)
    keep = min(k_s, tile, share)
    for layout in ("random", "skewed", "sparse"):
        per = []
        for t in range(tiles_s):
            n = tile if layout != "sparse" else int(rng.integers(0, 64))
            s = rng.standard_normal(n).astype(np.float32)
            if layout == "skewed" and t < 2:
                s += 8.0  # the first tiles hold every large score
            per.append(np.sort(ord_key(s))[::-1])
        sample = np.sort(np.concatenate(per))[::-1]
        kept = np.sort(np.concatenate([p[:keep] for p in per]))[::-1]
        thr_kept = int(kept[k_s - 1]) if len(kept) >= k_s else 0
        thr_sample = int(sample[k_s - 1]) if len(sample) >= k_s else 0
        assert thr_kept <= thr_sample
        top = sample[:k_s]
        crowded = any(int(np.count_nonzero(p >= top[-1])) > keep for p in per) if len(sample) >= k_s else False
        if not crowded and len(kept) >= k_s:
            assert thr_kept == thr_sample, layout
        if layout == "random":
            assert not crowded  # an even spread never fills four times a tile's share


@pytest.mark.parametrize("tiles,k", [(74, 5000), (244, 1000), (244, 4096), (1221, 20000), (78, 20000)])
def test_sampled_threshold_rarely_lets_fewer_than_k_through(tiles, k):
    """The wide-k first pass takes the k_s-th best of the first tiles / 16
    tiles, k_s = 1.5 k tiles_s / tiles + 32, as the starting threshold; a query
    falls back (runs again with none) when fewer than k documents of the whole
    collection reach it. On a collection in random slot order, the sample's
    k_s-th best is the k_s-th largest of n_s uniform draws (a Beta order
    statistic of the score distribution, whatever it is), and each of the other
    documents reaches it with probability 1 minus that quantile. Over 200,000
    draws of both, the documents that reach it sit at least 4.5 standard
    deviations above k and none of the draws falls short: about 1.5 k pass,
    so the fallback pass is for collections whose first slots are not a fair
    sample."""
    tile = 4096
    ts = tiles // 16
    n_s, n = ts * tile, tiles * tile
    k_s = (3 * k * ts + 2 * tiles - 1) // (2 * tiles) + 32
    rng = np.random.default_rng(tiles * 7 + k)
    trials = 200_000
    # the k_s-th largest of n_s uniforms is 1 - Beta(k_s, n_s - k_s + 1)
    tail = rng.beta(k_s, n_s - k_s + 1, trials)
    passing = k_s + rng.binomial(n - n_s, tail)
    assert passing.min() >= k, (passing.min(), k)
    z = (passing.mean() - k) / passing.std()
    assert z >= 4.5, z
    assert 1.4 * k <= passing.mean() <= 2.4 * k, passing.mean() / k
