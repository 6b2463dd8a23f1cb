"""A host model of the per-tile radix select (the most-significant-bit-first
walk over 32-bit score keys that the scoring kernels run on wavefront ballots)
against a brute-force sort, and of a variant that starts below the leading
bits every valid key shares (found from the largest and the smallest valid
key): both find the k-th largest key on random key sets with invalid (zero)
keys, ties, one sign only (the keys of non-negative scores all carry the top
bit) and mixed signs. Only the order-preserving key map of snn_device.h is
shared with the library; the walk is restated here."""
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
