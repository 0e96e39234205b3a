"""Host-side check of the index arithmetic behind the column passes' handling
of negligible classes (no GPU).  A forward column tile of compiled side M
with nthr threads stores element tid + j*nthr; the paired inverse tile loads
two runs of columns (k = p0 .. p0+P-1, then their partners M/2 - k in
memory order).  The kernels look up one flag per distinct value of
ky mod M/2 and per column (or pair); here every element of every thread is
compared with the class index the plain fold gives.  The tile geometry is
restated from the FP32 defaults: 4096 complex elements per workgroup,
8 per thread."""
import pytest


def fold(k, M):
    H, M4 = M // 2, M // 4
    return k if k <= M4 else (H - k if k <= H else (k - H if k <= H + M4 else M - k))


def shape_ok(MS, NT):
    return NT <= MS and MS % NT == 0 and ((MS // 2) % NT == 0 or NT % (MS // 2) == 0)


def fwd_geom(M):
    cols = max(4096 // M, 1)
    return cols, (cols * M + 7) // 8


def inv_geom(M):
    cols = max(4096 // M, 1)
    pcols = cols & ~1 if cols >= 2 else 2
    return pcols // 2, (pcols * M + 7) // 8


@pytest.mark.parametrize("M", [128, 192, 256, 384, 512, 768, 1024, 2048])
def test_forward_tile_flags(M):
    cols, NT = fwd_geom(M)
    H = M // 2
    if not shape_ok(M, NT):
        assert M not in (512, 1024, 2048)
        return
    CPT, U = M // NT, (H // NT if NT <= H else 1)
    assert cols * CPT <= 16
    for tid in range(NT):
        us = [fold((tid + v * NT) % H, M) for v in range(U)]
        for q in range(cols):
            for k in range(CPT):
                e = tid + (q * CPT + k) * NT
                assert e // M == q
                assert fold(e - q * M, M) == us[k % U]


@pytest.mark.parametrize("M", [512, 1024, 2048])
def test_inverse_tile_flags(M):
    P, NT = inv_geom(M)
    H = M // 2
    assert shape_ok(M, NT)
    CPT, U = M // NT, (H // NT if NT <= H else 1)
    F = P * CPT
    npair = H // 2 + 1
    for p0 in range(0, npair - P + 1, max(1, (npair - P) // 7)):
        c2 = H - p0 - P + 1
        for tid in range(NT):
            us = [fold((tid + v * NT) % H, M) for v in range(U)]
            for j in range(2 * F):
                e = tid + j * NT
                if j < F:
                    col, ky, pair = p0 + e // M, e % M, j // CPT
                else:
                    e2 = e - P * M
                    cm = (j - F) // CPT
                    col, ky, pair = c2 + cm, e2 - cm * M, P - 1 - cm
                # the pair's class row is the column's, and the row's class
                # index is the flag the thread loaded for it
                assert fold(col, M) == fold(p0 + pair, M)
                assert fold(ky, M) == us[(j % CPT) % U]


# LDS padding of the FFT stages: element i lives at i + i // 32.  A stage
# reads positions ib + r NB and writes ob + r NS (ob = t BSTRIDE + q NS R + k,
# k < NS); where the predicates below hold, the kernels use the padded base
# plus r S + (r S) // 32 instead of padding every position.
P = 32


def pad(i):
    return i + i // P


def linear_read(NB):
    return NB % P == 0


def linear_write(NS, R, B):
    return NS % P == 0 or (P % NS == 0 and ((NS * R) % P == 0 or P % (NS * R) == 0) and B % P == 0)


@pytest.mark.parametrize("L", [16, 24, 48, 64, 72, 96, 128, 192, 216, 256, 384, 512, 768, 1024, 2048])
def test_padded_lds_offsets(L):
    checked = 0
    for R in (2, 3, 4, 8):
        for NS in (1, 2, 3, 4, 6, 8, 9, 12, 16, 24, 27, 32, 48, 64, 72, 96, 128, 256, 512):
            if L % (NS * R):
                continue
            NB = L // R
            for B in (L, L + 2, 2 * L):
                for t in (0, 1, 3):
                    for j in range(0, NB, max(1, NB // 64)):
                        if linear_read(NB):
                            ib = t * B + j
                            for r in range(R):
                                assert pad(ib + r * NB) == pad(ib) + r * NB + (r * NB) // P
                                checked += 1
                        if linear_write(NS, R, B):
                            q, k = divmod(j, NS)
                            ob = t * B + q * NS * R + k
                            for r in range(R):
                                assert pad(ob + r * NS) == pad(ob) + r * NS + (r * NS) // P
                                checked += 1
    assert checked > 0 or L in (24, 72, 216)
