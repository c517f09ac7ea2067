"""Host check of the index mapping of the fused backward-row + accumulation gradient kernel.

For a batch of X-shifts that share their top bit j (and, when j >= nl, their bits above nl), the
kernel assigns row ch of the folded vector the x-side entries x(c) = c with a 0 inserted at bit j,
c = ch * 2^nl + p, written as (ins0(ch, j - nl) << nl) | p (j >= nl) or (ch << (nl + 1)) | ins0(p, j)
(j < nl), and the partner entries x(c) ^ a at block position p ^ m with m = a mod 2^nl (j >= nl) or
a mod 2^j (j < nl).  This test checks those formulas against the definition x(c), x(c) ^ a for every
row, position and shift of each qualifying batch shape, and that distinct rows never share an
entry (so the kernel needs no atomics)."""
import pytest


def ins0(c, j):
    return ((c >> j) << (j + 1)) | (c & ((1 << j) - 1))


def default_nl(nf):
    # default two-pass split for these sizes: half the folded bits in the row pass
    return (nf + 1) // 2


@pytest.mark.parametrize("n", [12, 13, 14, 16])
def test_fused_gradient_rows_own_disjoint_entries(n):
    nf = n - 1
    nl = default_nl(nf)
    nh = nf - nl
    row = 1 << nl
    batch = min(1 << nl, 64)
    checked = 0
    starts = list(range(batch, 1 << n, batch))
    for a0 in starts[:: max(1, len(starts) // 12)]:  # batch shapes spread over all top bits
        a_first, a_last = a0, a0 + batch - 1
        j = a_first.bit_length() - 1
        if a_last.bit_length() - 1 != j or (j >= nl and (a_first >> nl) != (a_last >> nl)):
            continue
        checked += 1
        jhi = j >= nl
        ah = a_first >> nl
        owner = {}
        for a in (a_first, a_last):
            m = (a & (row - 1)) if jhi else (a & ((1 << j) - 1))
            for ch in range(1 << nh):
                xh = ins0(ch, j - nl) if jhi else 0
                for p in range(row):
                    x_def = ins0(ch * row + p, j)
                    x = ((xh << nl) | p) if jhi else ((ch << (nl + 1)) | ins0(p, j))
                    assert x == x_def
                    q = p ^ m
                    y = (((xh ^ ah) << nl) | q) if jhi else ((ch << (nl + 1)) | ins0(q, j) | (1 << j))
                    assert y == x_def ^ a
                    for t in (x, y):
                        assert owner.setdefault(t, ch) == ch
        assert len(owner) == 1 << n  # every entry has exactly one owning row
    assert checked > 0


@pytest.mark.parametrize("nl", [6, 8, 9, 10])
@pytest.mark.parametrize("rb", [3, 4])
def test_fused_gradient_reads_the_row_pass_column_permutation(nl, rb):
    """The row pass (2^4-value register tiles) stores register r4 of thread t4, row position
    r4 + 16 t4, at column r4 2^(nl-4) + t4.  The fused kernel with 2^rb-value tiles wants register r
    of thread t at position r + 2^rb t and reads column (P mod 16) 2^(nl-4) + P / 16 for it: every
    column is read once and holds the position the kernel expects."""
    rbw = 4
    at = {}
    for t4 in range(1 << (nl - rbw)):
        for r4 in range(1 << rbw):
            at[(r4 << (nl - rbw)) | t4] = r4 + (t4 << rbw)
    seen = set()
    for t in range(1 << (nl - rb)):
        for r in range(1 << rb):
            p = r + (t << rb)
            col = ((p & ((1 << rbw) - 1)) << (nl - rbw)) | (p >> rbw)
            assert at[col] == p
            seen.add(col)
    assert seen == set(range(1 << nl))
