"""A second, independent Philox4x32-10 written with numpy column arithmetic.

Used only to cross-check the oracle's C implementation word for word.  The
round function and constants follow Salmon et al., SC'11: counter words 0 and
2 are multiplied by 0xD2511F53 and 0xCD9E8D57, the high product halves are
xor-ed with counter words 1 and 3 and the round key, and the key advances by
0x9E3779B9 and 0xBB67AE85 between rounds.
"""
import numpy as np

_MASK = np.uint64(0xFFFFFFFF)
_SHIFT = np.uint64(32)


def philox4x32(ctr, key, rounds=10):
    """ctr: (n, 4) uint32, key: (n, 2) uint32 -> (n, 4) uint32."""
    c = np.asarray(ctr, dtype=np.uint64).reshape(-1, 4)
    k = np.asarray(key, dtype=np.uint64).reshape(-1, 2)
    a, b, cc, d = (c[:, 0].copy(), c[:, 1].copy(), c[:, 2].copy(), c[:, 3].copy())
    ka, kb = k[:, 0].copy(), k[:, 1].copy()
    for r in range(rounds):
        if r:
            ka = (ka + np.uint64(0x9E3779B9)) & _MASK
            kb = (kb + np.uint64(0xBB67AE85)) & _MASK
        prod_a = a * np.uint64(0xD2511F53)
        prod_c = cc * np.uint64(0xCD9E8D57)
        a, b, cc, d = ((prod_c >> _SHIFT) ^ b ^ ka,
                       prod_c & _MASK,
                       (prod_a >> _SHIFT) ^ d ^ kb,
                       prod_a & _MASK)
    return np.stack([a, b, cc, d], axis=1).astype(np.uint32)
