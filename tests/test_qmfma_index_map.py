"""Host emulation of the index maps of the matrix-core M2L kernel (k_m2l_qmfma): every LDS read of
the rotation blocks (A operands, forward and transposed), every register slot, source role and
accumulator offset stays inside its buffer for every order, part, block, k-step and lane, and the
tile's LDS layout fits -- the same formulas as the kernel, evaluated on the CPU (no GPU needed)."""
import pytest


def S(n):
    return n // 4 + 1


def hoff(n):
    return sum(S(k) for k in range(n))


def rot_block_off(n):
    return n * (2 * n * n + 1) // 3


LDS_MAX = 163840


@pytest.mark.parametrize("P", [20, 22, 23, 24])
def test_qmfma_index_map_in_bounds(P):
    RS = P * (2 * P * P + 1) // 3
    assert RS == rot_block_off(P)
    NQ = hoff(P); NQP = (NQ + 1) // 2 * 2; P2 = P * P
    fixed = 8 * RS + 2 * 65 + 64
    per = 8 * 2 * P2 + 2 * (189 + 64) + 16
    NS = min(16, (LDS_MAX - fixed) // per)
    tb = 8 * (RS + NS * 2 * P2) + 4 * 4 * NS + 2 * (65 + 64 * NS + 189 * NS)
    assert NS >= 1 and tb <= LDS_MAX, (P, NS, tb)
    NB = (P + 15) // 16
    nA = 0
    for n in range(P):
        nbk = (n + 1 + 15) // 16; nst = (n + 1 + 3) // 4
        assert nst == S(n) and nbk <= NB
        for p in (0, 1):
            base = rot_block_off(n) + ((n + 1) ** 2 if p else 0)
            ld = n if p else n + 1
            size = n * n if p else (n + 1) ** 2
            for back in (False, True):
                for s in range(nst):
                    assert hoff(n) + s < NQ
                    for b in range(nbk):
                        nA += 1
                        for lane in range(64):
                            ai, ak = lane & 15, lane >> 4
                            mo, mi = 16 * b + ai, 4 * s + ak
                            r, c = (mi, mo) if back else (mo, mi)
                            ok = r <= n and c <= n and (p == 0 or (r >= 1 and c >= 1))
                            at = ((r - 1) * ld + (c - 1) if p else r * ld + c) if ok else 0
                            assert 0 <= at and (not ok or at < size), (P, n, p, r, c)
                            assert 0 <= base + at < RS
            for jj in range(S(n)):
                assert jj // 4 < nbk or (jj // 4 < NB), (P, n, jj)
                assert hoff(n) + jj < NQ
    # source loads: roles 8 pot + 4 part + k < 16, i < NQP/2
    for pot in (0, 1):
        for part in (0, 1):
            for k in range(4):
                role = 8 * pot + 4 * part + k
                assert role < 16 and (role * NQP + NQP - 1) < 16 * NQP
    # accumulation offsets within one potential's P^2 block
    for n in range(P):
        for k in range(4):
            for jj in range(S(n)):
                m = 4 * jj + k
                for okr in (True, False):
                    assert n * n + (m if okr else 0) < P2 or not okr or m > n
                    assert n * n + n + (m if (okr and m > 0) else 0) < P2 or m > n
