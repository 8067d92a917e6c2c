"""The library's pivoting blocks, as its C header documents them.

With RMGE_PIVOT_BLOCK the library stops the block recursion at panels of
`block` columns (the last may be narrower) and cuts a panel wider than 128 into
its first 128 columns and the rest.  The oracle takes any partition as an
argument; the tests that compare with the library pass it this one.
"""


def library_blocks(n, block):
    """Ends of the library's diagonal pivoting blocks for panels of `block`."""
    ends = []
    for s in range(0, n, block):
        b = min(block, n - s)
        if b > 128:
            ends.append(s + 128)
        ends.append(s + b)
    return ends


def spans(ends):
    """[(start, end)] of consecutive blocks from their ends."""
    out, s = [], 0
    for e in ends:
        out.append((s, e))
        s = e
    return out
