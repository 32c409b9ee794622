"""The ordering fact behind the device's lexicographic sort of strings with
few bit transitions, checked on the CPU against the oracle's order (no GPU):
read the varying words of a string as one bit string, most significant bit
first, with a 0 above it; with G_j the place (0 at the top) of the j-th bit
that differs from the bit above it and L the number of bits, the codes
c_j = L - G_j (odd j) and c_j = G_j (even j), a missing transition taking 0
(odd j) or L (even j), compare as tuples exactly as the strings compare.
The codes here are computed from that definition, bit by bit."""
import numpy as np
import pytest

import synth
from oracle import lexorder as LX


def _bits(x, z, t, vary):
    """The bit string of term t over the varying word columns, most
    significant word and bit first (X[W-1] ... X[0], Z[W-1] ... Z[0])."""
    W = x.shape[1]
    out = []
    for col in vary:
        v = int(x[t, col - W]) if col >= W else int(z[t, col])
        out.extend((v >> (63 - i)) & 1 for i in range(64))
    return out


def _codes(bits, slots):
    L = len(bits)
    codes, prev = [], 0
    for g, b in enumerate(bits):
        if b != prev:
            j = len(codes) + 1
            codes.append(L - g if j % 2 else g)
            prev = b
    while len(codes) < slots:
        j = len(codes) + 1
        codes.append(0 if j % 2 else L)
    return tuple(codes)


def _case(kind, n, m, seed):
    rng = synth.rng_for(990, seed)
    if kind == "jw":
        x, z = synth.jordan_wigner(rng, n, m)
    else:
        d = synth.random_sum(rng, n, m, wmax=min(n, 4 if kind == "sparse" else n),
                             distinct_strings=False)
        x, z = d["x"], d["z"]
    W = x.shape[1]
    # repeats, a zero string, and strings differing only in their last bit
    x[1], z[1] = x[0], z[0]
    x[2], z[2] = 0, 0
    x[3], z[3] = x[0], z[0] ^ np.uint64(1)
    if n >= 64 and kind != "jw":
        z[4, 0] = np.uint64(0xFFFFFFFFFFFFFFFF)  # a word of ones
    return x, z


@pytest.mark.parametrize("kind,n,m", [("jw", 70, 300), ("jw", 200, 300), ("sparse", 130, 400),
                                      ("dense", 40, 300), ("dense", 64, 200), ("sparse", 1000, 200)])
def test_transition_codes_order_as_the_strings(kind, n, m):
    x, z = _case(kind, n, m, n + m)
    W = x.shape[1]
    cols = list(range(2 * W - 1, W - 1, -1)) + list(range(W - 1, -1, -1))  # X high..low, Z high..low
    vary = [c for c in cols
            if np.unique(x[:, c - W] if c >= W else z[:, c]).size > 1]
    bit_rows = [_bits(x, z, t, vary) for t in range(m)]
    slots = max(sum(1 for g in range(len(b)) if b[g] != (b[g - 1] if g else 0)) for b in bit_rows)
    keys = [_codes(b, slots) for b in bit_rows]
    mine = sorted(range(m), key=lambda t: keys[t])  # stable
    assert list(LX.order(x, z)) == mine
