"""Hilbert space-filling-curve index (oracle).

The paper orders coarse cells (Alg. 1, step 2) and orbital centres (Alg. 2,
step 3) along a Hilbert curve without naming the variant.  This oracle takes
J. Skilling's transform ("Programming the Hilbert curve", AIP Conf. Proc.
707, 2004): the axes-to-transpose map undoes the excess work of the
inverse Gray code bit plane by bit plane, Gray-encodes, and the index is the
transposed form read with the most significant bit plane first and axis 0
first within a plane.  Axis 0 is x, 1 is y, 2 is z.
"""

from __future__ import annotations


def hilbert_index(coords, bits: int) -> int:
    """Hilbert index of the integer point ``coords`` in a 2^bits cube."""
    x = [int(c) for c in coords]
    nd = len(x)
    if bits < 1:
        raise ValueError("bits must be >= 1")
    for c in x:
        if c < 0 or c >= (1 << bits):
            raise ValueError("coordinate outside the cube")
    top = 1 << (bits - 1)
    # undo excess work, from the top bit plane down to bit 1
    q = top
    while q > 1:
        low = q - 1
        for i in range(nd):
            if x[i] & q:
                x[0] ^= low              # invert the low bits of axis 0
            else:
                t = (x[0] ^ x[i]) & low  # exchange low bits of axes 0 and i
                x[0] ^= t
                x[i] ^= t
        q >>= 1
    # Gray encode
    for i in range(1, nd):
        x[i] ^= x[i - 1]
    t = 0
    q = top
    while q > 1:
        if x[nd - 1] & q:
            t ^= q - 1
        q >>= 1
    for i in range(nd):
        x[i] ^= t
    # read the transposed form: bit plane by plane, axis 0 first
    h = 0
    for b in range(bits - 1, -1, -1):
        for i in range(nd):
            h = (h << 1) | ((x[i] >> b) & 1)
    return h


def bits_for(extent: int) -> int:
    """Smallest b >= 1 with 2^b >= extent."""
    b = 1
    while (1 << b) < extent:
        b += 1
    return b
