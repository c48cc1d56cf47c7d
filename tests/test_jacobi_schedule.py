"""The pair schedule of the one-sided Jacobi sweep (m <= 128 kernel) and the
steps at which it needs a workgroup barrier.

A sweep visits the pairs (i, i ^ k), k = 1 .. M-1, grouped by the top bit h
of k; pair slot q keeps its lower column i (bit h clear) in registers over
its group, and the partner column goes through LDS.  Slot q runs on lanes
q*TPP .. q*TPP + TPP - 1, TPP = min(2*256/M, M).  The kernel puts a
workgroup barrier after step k of a group only when (k + 1) is a multiple of
the pair slots per wavefront, 64 / TPP (and after each group); the other steps
rely on one wavefront's LDS operations taking effect in order.  Brute force
over every pair and step: each partner read at step k + 1 whose writer at
step k sits in another wavefront is behind such a barrier, and every sweep
visits every pair exactly once."""
import pytest


def schedule(M, NT=256):
    TPP = min(2 * NT // M, M)
    return TPP, 64 // TPP


@pytest.mark.parametrize("M", [16, 32, 64, 128])
def test_cross_wavefront_dependencies_have_barriers(M):
    TPP, PSW = schedule(M)
    for h in range(M.bit_length() - 1):
        for k in range(1 << h, (2 << h) - 1):          # the group's last step is followed by a barrier
            barrier = (k + 1) % PSW == 0
            for q in range(M // 2):
                i = ((q >> h) << (h + 1)) | (q & ((1 << h) - 1))
                writer_lower = (i ^ (k + 1)) ^ k           # who rotated the partner at step k
                assert (writer_lower >> h) & 1 == 0
                qw = ((writer_lower >> (h + 1)) << h) | (writer_lower & ((1 << h) - 1))
                if (q * TPP) // 64 != (qw * TPP) // 64:
                    assert barrier, (M, h, k, q)


@pytest.mark.parametrize("M", [16, 32, 64, 128])
def test_sweep_visits_every_pair_once_and_barrier_count(M):
    TPP, PSW = schedule(M)
    seen = set()
    barriers = 0
    for h in range(M.bit_length() - 1):
        for k in range(1 << h, 2 << h):
            cols = set()
            for q in range(M // 2):
                i = ((q >> h) << (h + 1)) | (q & ((1 << h) - 1))
                j = i ^ k
                assert i < j and i not in cols and j not in cols
                cols |= {i, j}
                seen.add((i, j))
            barriers += (k + 1) % PSW == 0 and k + 1 < (2 << h)
        barriers += 1                                   # after the group
    assert len(seen) == M * (M - 1) // 2
    assert barriers == {16: 5, 32: 9, 64: 10, 128: 11}[M]


@pytest.mark.parametrize("M", [16, 32, 64, 128])
def test_fp32_width_change_never_overwrites_unread_values(M):
    """The BF16 path rotates in FP32: L (double columns at stride LDB) is
    narrowed in place to float columns at stride LDF = M + TPP by chunks of
    CC columns in increasing order (each chunk reads all its doubles, then a
    barrier, then writes its floats), and widened back in decreasing order.
    No chunk's writes may reach bytes a later chunk still reads, and the float
    columns must stay inside the double array."""
    NT = 256
    TPP, _ = schedule(M, NT)
    LDB, LDF = M + min(TPP, 8), M + TPP
    CC = M if M * M // NT <= 16 else 16 * NT // M
    assert M % CC == 0 and (CC * M) % NT == 0 and CC * M // NT <= 16

    def dbl(c):
        return (8 * c * LDB, 8 * c * LDB + 8 * M)

    def flt(c):
        return (4 * c * LDF, 4 * c * LDF + 4 * M)

    def overlap(a, b):
        return a[0] < b[1] and b[0] < a[1]

    chunks = [range(c0, c0 + CC) for c0 in range(0, M, CC)]
    for j, ch in enumerate(chunks):
        for later in chunks[j + 1:]:           # narrowing: later chunks read doubles
            assert not any(overlap(flt(c), dbl(c2)) for c in ch for c2 in later)
        for earlier in chunks[:j]:             # widening runs downward: lower chunks read floats
            assert not any(overlap(dbl(c), flt(c2)) for c in ch for c2 in earlier)
    assert flt(M - 1)[1] <= 8 * M * LDB
