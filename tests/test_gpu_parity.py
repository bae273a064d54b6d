"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances (FP64 everywhere on this path): residuals and single contractions
1e-11 absolute on O(1) values (rounding of sums with up to a few thousand
terms); converged energies 1e-8 Eh and amplitudes 1e-7 (the convergence
threshold 1e-8 on ||dT||, both sides converge independently); the (T) energy
of given amplitudes 1e-11 relative.
"""
import ctypes as C
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2407_11258_amd import lnocc as L  # noqa: E402
from oracle import ccsd as occ, triples as otr  # noqa: E402
from synth import make_fragment  # noqa: E402

DEV = "cuda:0"


def say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _random_amplitudes(o, v, seed, scale=0.05):
    rng = np.random.default_rng(seed)
    t1 = scale * rng.standard_normal((o, v))
    t2 = scale * rng.standard_normal((o, o, v, v))
    return t1, t2 + t2.transpose(1, 0, 3, 2)


# ------------------------------------------------------------ contraction kernel
_KEEP = []   # device tensors referenced by raw pointers must outlive the call


def _operand(t, ro, ri, ko, ki, b0=0, b1=0, bid=0):
    _KEEP.append(t)
    return L.lnocc_operand_t(t.data_ptr(), ro, ri, ko, ki, b0, b1, bid)


def _contract(M, Mi, N, Ni, c, cstr, segs, beta=0.0, batch=1, nb1=1, cb=(0, 0, 0), precision=0,
              tile=0):
    d = L.lnocc_contract_t()
    d.M, d.Mi, d.N, d.Ni = M, Mi, N, Ni
    d.nseg = len(segs)
    for s, (K, Ki, scale, a, b) in enumerate(segs):
        d.K[s], d.Ki[s], d.scale[s] = K, Ki, scale
        d.a[s], d.b[s] = a, b
    d.c = c.data_ptr()
    d.c_mo, d.c_mi, d.c_no, d.c_ni = cstr
    d.c_b0, d.c_b1, d.c_bid = cb
    d.beta, d.batch, d.nb1 = beta, batch, nb1
    d.precision = precision
    d.tile = tile
    st = L.lnocc_contract(d, torch.cuda.current_stream().cuda_stream)
    _KEEP.clear()
    assert st == L.LNOCC_OK, f"{L.lnocc_status_string(st)}: {L.lnocc_last_error()}"


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (130, 70, 37), (257, 129, 200), (64, 300, 5)])
def test_contract_plain_and_transposed(M, N, K):
    say(f"contract plain M={M} N={N} K={K}")
    rng = np.random.default_rng(M + N + K)
    A = rng.standard_normal((M, K))
    Bm = rng.standard_normal((N, K))
    ref = A @ Bm.T
    c = torch.zeros((M, N), dtype=torch.float64, device=DEV)
    # operands contiguous along k
    _contract(M, 1, N, 1, c, (N, 0, 1, 0),
              [(K, 1, 1.0, _operand(dev(A), K, 0, 1, 0), _operand(dev(Bm), K, 0, 1, 0))])
    np.testing.assert_allclose(host(c), ref, rtol=0, atol=1e-12 * max(1, K))
    # operands contiguous along the row index (stored transposed), C transposed
    At, Bt = dev(A.T.copy()), dev(Bm.T.copy())
    ct = torch.zeros((N, M), dtype=torch.float64, device=DEV)
    _contract(M, 1, N, 1, ct, (1, 0, M, 0),
              [(K, 1, 1.0, _operand(At, 1, 0, M, 0), _operand(Bt, 1, 0, N, 0))])
    np.testing.assert_allclose(host(ct).T, ref, rtol=0, atol=1e-12 * max(1, K))


def test_contract_two_index_modes_segments_and_batch():
    say("contract two-index modes, segments, batch")
    o, v, nb0, nb1 = 5, 19, 2, 3
    rng = np.random.default_rng(3)
    T = rng.standard_normal((nb0, o, o, v, v))      # T[e0][k][i][a][c]
    U = rng.standard_normal((nb1, o, o, v, v))      # U[e1][k][j][b][c]
    P = rng.standard_normal((v, 7))                 # second segment: sum_e P[a, e] Q[b, e]
    Qm = rng.standard_normal((v, 7))
    C0 = rng.standard_normal((nb0 * nb1, o, o, v, v))
    ref = np.einsum("xkiac,ykjbc->xyijab", T, U).reshape(nb0 * nb1, o, o, v, v)
    ref = ref - 0.5 * np.einsum("ae,be->ab", P, Qm)[None, None, None] + 2.0 * C0
    c = dev(C0)
    ovv, vv = o * v * v, v * v
    # m = (i, a), n = (j, b), k = (k, c); C[e][i][j][a][b]
    seg1 = (o * v, v, 1.0,
            _operand(dev(T), vv, v, ovv, 1, b0=o * ovv),
            _operand(dev(U), vv, v, ovv, 1, b1=o * ovv))
    # the same C for every (i, j) pair: rows (i, a) with zero stride on i
    seg2 = (7, 1, -0.5, _operand(dev(P), 0, 7, 1, 0), _operand(dev(Qm), 0, 7, 1, 0))
    _contract(o * v, v, o * v, v, c, (ovv, v, vv, 1), [seg1, seg2], beta=2.0,
              batch=nb0 * nb1, nb1=nb1, cb=(0, 0, o * ovv))
    np.testing.assert_allclose(host(c), ref, rtol=0, atol=1e-11)


def _bf16_round(x):
    """Round to the nearest bf16 (ties to even) and return (bits, value)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    bits = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    val = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return bits, val


@pytest.mark.parametrize("M,N,K", [(130, 70, 37), (257, 160, 200), (20, 33, 1000)])
def test_contract_low_precision(M, N, K):
    say(f"contract fp32/bf16 M={M} N={N} K={K}")
    rng = np.random.default_rng(7 + M)
    A = rng.standard_normal((M, K))
    Bm = rng.standard_normal((N, K))
    # FP32: operands exactly representable, FP32 accumulation
    A32, B32 = A.astype(np.float32), Bm.astype(np.float32)
    ref = A32.astype(np.float64) @ B32.astype(np.float64).T
    c = torch.zeros((M, N), dtype=torch.float64, device=DEV)
    a_t = torch.tensor(A32, device=DEV)
    b_t = torch.tensor(B32, device=DEV)
    _contract(M, 1, N, 1, c, (N, 0, 1, 0),
              [(K, 1, 1.0, _operand(a_t, K, 0, 1, 0), _operand(b_t, K, 0, 1, 0))], precision=1)
    err = np.abs(host(c) - ref).max() / np.abs(ref).max()
    assert err < 2e-6 * np.sqrt(K), err
    # BF16: operands rounded to bf16 on the host, FP32 accumulation; also the
    # row-contiguous (transposed) operand layout
    abits, aval = _bf16_round(A)
    bbits, bval = _bf16_round(Bm)
    ref = aval @ bval.T
    a_t = torch.tensor(abits.T.copy().view(np.int16), device=DEV)
    b_t = torch.tensor(bbits.view(np.int16), device=DEV)
    c.zero_()
    _contract(M, 1, N, 1, c, (N, 0, 1, 0),
              [(K, 1, 1.0, _operand(a_t, 1, 0, M, 0), _operand(b_t, K, 0, 1, 0))], precision=2)
    err = np.abs(host(c) - ref).max() / np.abs(ref).max()
    assert err < 2e-6 * np.sqrt(K), err


@pytest.mark.parametrize("tile", [1, 2, 3, 4, 5, 6, 7, 8, 9])
@pytest.mark.parametrize("precision", [0, 1])
def test_contract_every_tile(tile, precision):
    """Each tile shape of the launcher (forced) on a ragged, segmented, two-index
    product, FP64 and FP32 operands, both operands once contiguous along k and
    once along their row index (the 128x160 and 256x128 tiles and the split bf16
    products of tiles 7 and 9 are for FP32 operands only, the 160x160 tile for FP64
    only; otherwise the automatic choice runs)."""
    say(f"contract tile {tile} precision {precision}")
    rng = np.random.default_rng(100 + tile)
    M, N, K1, K2 = 301, 263, 45, 19
    A1, B1 = rng.standard_normal((M, K1)), rng.standard_normal((N, K1))
    A2, B2 = rng.standard_normal((K2, M)), rng.standard_normal((K2, N))
    dt = np.float64 if precision == 0 else np.float32
    A1, B1, A2, B2 = (x.astype(dt) for x in (A1, B1, A2, B2))
    ref = (A1.astype(np.float64) @ B1.astype(np.float64).T
           - 0.5 * A2.astype(np.float64).T @ B2.astype(np.float64))
    c = torch.zeros((M, N), dtype=torch.float64, device=DEV)
    t = [torch.tensor(x, device=DEV) for x in (A1, B1, A2, B2)]
    _contract(M, 1, N, 1, c, (N, 0, 1, 0),
              [(K1, 1, 1.0, _operand(t[0], K1, 0, 1, 0), _operand(t[1], K1, 0, 1, 0)),
               (K2, 1, -0.5, _operand(t[2], 1, 0, M, 0), _operand(t[3], 1, 0, N, 0))],
              precision=precision, tile=tile)
    err = np.abs(host(c) - ref).max() / np.abs(ref).max()
    assert err < (1e-13 if precision == 0 else 2e-6 * np.sqrt(K1 + K2)), err


@pytest.mark.parametrize("shift", [0, 1])
@pytest.mark.parametrize("tile", [1, 2, 3, 4, 5, 6, 7, 8, 9])
@pytest.mark.parametrize("precision", [0, 1])
def test_contract_column_major_output(tile, precision, shift):
    """Outputs whose row index is the contiguous one (C[e][n][mo][mi]), read and
    written back with beta != 0: with shift = 0 every 4-row group is one aligned
    vector, so the kernels store it at once (FP64 accumulators after a lane
    exchange); shift = 1 misaligns C by one element and takes the element-wise
    path.  Ragged in M and N, batched, every tile."""
    say(f"contract column-major C tile {tile} precision {precision} shift {shift}")
    rng = np.random.default_rng(300 + 10 * tile + precision)
    nb, Mo, Mi, N, K = 2, 7, 36, 263, 53
    M = Mo * Mi
    dt = np.float64 if precision == 0 else np.float32
    A = rng.standard_normal((nb, M, K)).astype(dt)
    Bm = rng.standard_normal((nb, N, K)).astype(dt)
    C0 = rng.standard_normal((nb, N, M))
    ref = 0.75 * C0 + np.einsum("emk,enk->enm", A.astype(np.float64), Bm.astype(np.float64))
    buf = torch.zeros(nb * N * M + shift, dtype=torch.float64, device=DEV)
    c = buf[shift:]
    c.copy_(torch.tensor(C0.ravel(), device=DEV))
    a_t, b_t = torch.tensor(A, device=DEV), torch.tensor(Bm, device=DEV)
    _contract(M, Mi, N, 1, c, (Mi, 1, M, 0),
              [(K, 1, 1.0, _operand(a_t, Mi * K, K, 1, 0, bid=M * K),
                _operand(b_t, K, 0, 1, 0, bid=N * K))],
              beta=0.75, batch=nb, cb=(0, 0, N * M), precision=precision, tile=tile)
    got = host(c).reshape(nb, N, M)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err < (1e-14 if precision == 0 else 2e-6 * np.sqrt(K)), err


@pytest.mark.parametrize("M,Mi,K,kfast", [(20, 1, 7, False), (5000, 100, 333, False),
                                          (40000, 1, 64, False), (37, 1, 1000, True),
                                          (3000, 30, 2560, True)])
def test_contract_matrix_vector(M, Mi, K, kfast):
    """N = 1 (FP64, one segment) runs the matrix-vector kernels: rows contiguous
    (block of rows x interleaved k streams) or k contiguous (one wave per row),
    with a two-index row mode and beta != 0."""
    say(f"contract matrix-vector M={M} Mi={Mi} K={K} kfast={kfast}")
    rng = np.random.default_rng(M + K)
    A = rng.standard_normal((M, K))
    x = rng.standard_normal(K)
    C0 = rng.standard_normal(M)
    ref = 0.5 * (A @ x) - 1.5 * C0
    Mo = M // Mi
    if kfast:   # A[m][k], m = (mo, mi)
        a_t = dev(A)
        op = _operand(a_t, Mi * K, K, 1, 0)
    else:       # stored as A^T[k][m]
        a_t = dev(A.T.copy())
        op = _operand(a_t, Mi, 1, M, 0)
    xb = dev(x)
    src = dev(C0)
    c = torch.full((M,), float("nan"), dtype=torch.float64, device=DEV)
    d = L.lnocc_contract_t()
    d.M, d.Mi, d.N, d.Ni = M, Mi, 1, 1
    d.nseg = 1
    d.K[0], d.Ki[0], d.scale[0] = K, 1, 0.5
    d.a[0], d.b[0] = op, _operand(xb, 0, 0, 1, 0)
    d.c = c.data_ptr()
    d.c_mo, d.c_mi, d.c_no, d.c_ni = Mi, 1, 0, 0
    d.beta, d.batch, d.nb1, d.precision = -1.5, 1, 1, 0
    # the beta input comes from C itself through the ABI: copy it in first
    c.copy_(src)
    st = L.lnocc_contract(d, torch.cuda.current_stream().cuda_stream)
    _KEEP.clear()
    assert st == L.LNOCC_OK, L.lnocc_last_error()
    np.testing.assert_allclose(host(c), ref, rtol=0, atol=1e-12 * np.sqrt(K) * np.abs(ref).max())


@pytest.mark.parametrize("tile,precision", [(0, 3), (1, 3), (2, 3), (3, 3), (4, 3), (0, 4),
                                            (1, 4), (3, 4), (10, 3), (10, 4)])
def test_contract_split_products_exact(tile, precision):
    """Split bf16 products (LNOCC_FP32_SPLIT on FP32 operands, LNOCC_FP64_SPLIT
    on FP64 ones) on operands x = s (1 + c 2^-9), s = +-1, c in {-1, 0, 1}: x
    needs 10 significant bits (exact in FP32, so the FP64 -> FP32 rounding is
    exact too), so it splits into a bf16 high part s and a nonzero middle part
    s c 2^-9.  Every part product the kernel forms is exact, and with K = 16
    every partial sum fits FP32's 24 bits, so C must equal the exact product
    bit for bit; dropping the middle-part products (h m', m h', m m') would
    change it by multiples of 2^-18."""
    say(f"contract split products exact tile {tile} precision {precision}")
    rng = np.random.default_rng(40 + tile)
    M, N, K = (132, 72, 16) if tile >= 10 else (133, 70, 16)   # 4 x 4 staging: multiples of 4

    def draw(*shape):
        sgn = rng.choice([-1.0, 1.0], size=shape)
        return sgn * (1.0 + rng.integers(-1, 2, size=shape) * 2.0 ** -9)

    A, Bm = draw(M, K), draw(N, K)
    ref = A @ Bm.T                                   # exact in FP64 (<= 30 bits)
    c = torch.zeros((M, N), dtype=torch.float64, device=DEV)
    dt = np.float32 if precision == L.LNOCC_FP32_SPLIT else np.float64
    a_t = torch.tensor(A.astype(dt), device=DEV)
    b_t = torch.tensor(Bm.astype(dt), device=DEV)
    _contract(M, 1, N, 1, c, (N, 0, 1, 0),
              [(K, 1, 1.0, _operand(a_t, K, 0, 1, 0), _operand(b_t, K, 0, 1, 0))],
              precision=precision, tile=tile)
    np.testing.assert_array_equal(host(c), ref)


@pytest.mark.parametrize("tile", [10])
@pytest.mark.parametrize("precision", [1, 3, 4])
def test_contract_split_v4_layouts(precision, tile):
    """Tile 10 (split products staged as 4 x 4 blocks) on the layouts it takes:
    a k-contiguous operand with a two-index k (inner extent 36, padded row
    pitch) and two-index rows, a row-contiguous operand pair (4-row groups
    along memory), a batch of two, beta != 0, ragged M and N (multiples of 4,
    not of 128) and K not a multiple of the 32-k slice; FP32 operands (precision
    1 and 3) and FP64 operands (4).  FP32-level agreement with the FP64 product."""
    say(f"contract split v4 layouts precision {precision} tile {tile}")
    rng = np.random.default_rng(500 + precision)
    nb, o, v, Ko, Ki, N, K2 = 2, 4, 36, 5, 36, 132, 68
    M, K1 = o * v, Ko * Ki
    A1p = rng.standard_normal((nb, o, v, Ko, Ki + 4))    # rows (i, a), k = (x, c), padded pitch
    B1 = rng.standard_normal((nb, N, K1))
    A2 = rng.standard_normal((nb, K2, M))                # row-contiguous
    B2 = rng.standard_normal((nb, K2, N))
    C0 = rng.standard_normal((nb, M, N))
    dt = np.float64 if precision == 4 else np.float32
    A1p, B1, A2, B2 = (x.astype(dt) for x in (A1p, B1, A2, B2))
    A1 = A1p[..., :Ki].reshape(nb, M, K1).astype(np.float64)
    ref = (np.einsum("emk,enk->emn", A1, B1.astype(np.float64))
           - 0.25 * np.einsum("ekm,ekn->emn", A2.astype(np.float64), B2.astype(np.float64))
           + 0.5 * C0)
    tA1, tB1, tA2, tB2 = (torch.tensor(np.ascontiguousarray(x), device=DEV) for x in (A1p, B1, A2, B2))
    c = dev(C0)
    sri, sko = Ko * (Ki + 4), Ki + 4
    seg1 = (K1, Ki, 1.0, _operand(tA1, v * sri, sri, sko, 1, bid=o * v * sri),
            _operand(tB1, K1, 0, Ki, 1, bid=N * K1))
    seg2 = (K2, 1, -0.25, _operand(tA2, v, 1, M, 0, bid=K2 * M),
            _operand(tB2, 1, 0, N, 0, bid=K2 * N))
    _contract(M, v, N, 1, c, (N * v, N, 1, 0), [seg1, seg2], beta=0.5, batch=nb, nb1=1,
              cb=(0, 0, M * N), precision=precision, tile=tile)
    err = np.abs(host(c) - ref).max() / np.abs(ref).max()
    say(f"  relative error {err:.2e}")
    assert err < 2e-6 * np.sqrt(K1 + K2)


@pytest.mark.parametrize("tile", [0, 1, 3])
def test_contract_fp64_split_accuracy(tile):
    """LNOCC_FP64_SPLIT on full-mantissa FP64 operands (the arithmetic of the
    ring contractions in the reduced modes): each operand is rounded to FP32
    (relative error 2^-24) and split, so the result has FP32-level accuracy
    against the FP64 product; a row-contiguous second segment and beta."""
    say(f"contract FP64 split accuracy tile {tile}")
    rng = np.random.default_rng(80 + tile)
    M, N, K1, K2 = 299, 257, 640, 33
    A1, B1 = rng.standard_normal((M, K1)), rng.standard_normal((N, K1))
    A2, B2 = rng.standard_normal((K2, M)), rng.standard_normal((N, K2))
    C0 = rng.standard_normal((M, N))
    ref = A1 @ B1.T - 0.5 * A2.T @ B2.T + 0.25 * C0
    t = [dev(x) for x in (A1, B1, A2, B2)]
    segs = [(K1, 1, 1.0, _operand(t[0], K1, 0, 1, 0), _operand(t[1], K1, 0, 1, 0)),
            (K2, 1, -0.5, _operand(t[2], 1, 0, M, 0), _operand(t[3], K2, 0, 1, 0))]
    c = dev(C0)
    _contract(M, 1, N, 1, c, (N, 0, 1, 0), segs, precision=L.LNOCC_FP64_SPLIT, tile=tile,
              beta=0.25)
    err = np.abs(host(c) - ref).max() / np.abs(ref).max()
    say(f"  relative error {err:.2e}")
    assert err < 2e-6 * np.sqrt(K1 + K2)
    assert err > 1e-12          # not FP64 products


@pytest.mark.parametrize("tile", [0, 1, 3])
def test_contract_split_products_accuracy(tile):
    """Split bf16 products on full-mantissa FP32 operands: FP32-level accuracy
    (the representation error of the three parts is below 2^-27 and the dropped
    part products below 2^-24 of each product), far from what bf16 operands
    give on the same data.  Two segments, one with a row-contiguous operand."""
    say(f"contract split products accuracy tile {tile}")
    rng = np.random.default_rng(60 + tile)
    M, N, K1, K2 = 301, 263, 300, 37
    A1, B1 = rng.standard_normal((M, K1)), rng.standard_normal((N, K1))
    A2, B2 = rng.standard_normal((K2, M)), rng.standard_normal((N, K2))
    A1, B1, A2, B2 = (x.astype(np.float32) for x in (A1, B1, A2, B2))
    ref = (A1.astype(np.float64) @ B1.astype(np.float64).T
           + 0.25 * A2.astype(np.float64).T @ B2.astype(np.float64).T)
    t = [torch.tensor(x, device=DEV) for x in (A1, B1, A2, B2)]
    segs = [(K1, 1, 1.0, _operand(t[0], K1, 0, 1, 0), _operand(t[1], K1, 0, 1, 0)),
            (K2, 1, 0.25, _operand(t[2], 1, 0, M, 0), _operand(t[3], K2, 0, 1, 0))]
    errs = {}
    for prec in (L.LNOCC_FP32, L.LNOCC_FP32_SPLIT):
        c = torch.zeros((M, N), dtype=torch.float64, device=DEV)
        _contract(M, 1, N, 1, c, (N, 0, 1, 0), segs, precision=prec, tile=tile)
        errs[prec] = np.abs(host(c) - ref).max() / np.abs(ref).max()
    say(f"  relative error fp32 {errs[L.LNOCC_FP32]:.2e} split {errs[L.LNOCC_FP32_SPLIT]:.2e}")
    assert errs[L.LNOCC_FP32_SPLIT] < 2e-6 * np.sqrt(K1 + K2)
    assert errs[L.LNOCC_FP32_SPLIT] < 4 * errs[L.LNOCC_FP32] + 1e-7


# ------------------------------------------------------------ solver pieces
def _fragment_on_device(f, scale=1.0):
    return dev(scale * f.B), dev(f.eps_occ), dev(f.eps_vir)


def _call(fn, f, B, eo, ev, t1, t2, conv_tol=1e-8, **kw):
    opt = L.make_options(**kw)
    fs = L.make_fragment_struct(B, eo, ev, t1, t2, conv_tol)
    ws = L.Workspace(DEV)
    ws.attach([fs], opt)
    st = fn(fs, opt)
    if st < 0:
        say(f"  status {st}: {L.lnocc_last_error()}")
    return st, fs


@pytest.mark.parametrize("o,v,X,seed", [(3, 13, 40, 21), (2, 37, 61, 22), (5, 9, 17, 23)])
@pytest.mark.parametrize("ladder", ["stored", "on_the_fly"])
def test_residuals_match_oracle(o, v, X, seed, ladder):
    say(f"residuals o={o} v={v} X={X} ladder {ladder}")
    f = make_fragment(o, v, X, seed)
    t1, t2 = _random_amplitudes(o, v, seed)
    R1o, R2o = occ.residuals(2.0 * f.B, f.eps_occ, f.eps_vir, t1, t2)
    B, eo, ev = _fragment_on_device(f, 2.0)
    t1d, t2d = dev(t1), dev(t2)
    r1 = torch.empty((o, v), dtype=torch.float64, device=DEV)
    r2 = torch.empty((o, o, v, v), dtype=torch.float64, device=DEV)
    opt = L.make_options(ladder=ladder)
    fs = L.make_fragment_struct(B, eo, ev, t1d, t2d, 1e-8)
    ws = L.Workspace(DEV)
    ws.attach([fs], opt)
    st = L.lnocc_ccsd_residuals(fs, opt, r1.data_ptr(), r2.data_ptr())
    assert st == L.LNOCC_OK, L.lnocc_status_string(st)
    np.testing.assert_allclose(host(r1), R1o, rtol=0, atol=1e-11)
    np.testing.assert_allclose(host(r2), R2o, rtol=0, atol=1e-11)


@pytest.mark.parametrize("o,v,X,seed", [(3, 13, 40, 31), (4, 21, 50, 32), (1, 10, 20, 33)])
def test_triples_match_oracle(o, v, X, seed):
    say(f"triples o={o} v={v} X={X}")
    f = make_fragment(o, v, X, seed)
    t1, t2 = _random_amplitudes(o, v, seed, scale=0.1)
    ref = otr.e_triples_restricted(2.0 * f.B, f.eps_occ, f.eps_vir, t1, t2)
    B, eo, ev = _fragment_on_device(f, 2.0)
    st, fs = _call(L.lnocc_fragment_triples, f, B, eo, ev, dev(t1), dev(t2), triples_batch=3)
    assert st == L.LNOCC_OK, L.lnocc_status_string(st)
    if o == 1:
        assert fs.e_t == 0.0
    else:
        assert abs(fs.e_t - ref) < 1e-11 * max(1.0, abs(ref)), (fs.e_t, ref)


@pytest.mark.parametrize("o,v,X,seed,chunk", [(4, 20, 72, 0, 0), (6, 45, 100, 5, 45 ** 3 * 8 * 7),
                                              (2, 3, 5, 9, 0)])
def test_full_solve_matches_oracle(o, v, X, seed, chunk):
    say(f"full solve o={o} v={v} X={X} seed={seed}")
    f = make_fragment(o, v, X, seed)
    ref = occ.ccsd(f.B, f.eps_occ, f.eps_vir, conv_tol=1e-10)
    assert ref.converged
    ref_t = otr.e_triples_restricted(f.B, f.eps_occ, f.eps_vir, ref.t1, ref.t2)
    B, eo, ev = _fragment_on_device(f)
    t1 = torch.empty((o, v), dtype=torch.float64, device=DEV)
    t2 = torch.empty((o, o, v, v), dtype=torch.float64, device=DEV)
    st, fs = _call(L.lnocc_fragment_ccsd, f, B, eo, ev, t1, t2, conv_tol=1e-10,
                   ladder_chunk_bytes=chunk, ladder="on_the_fly" if chunk else "stored")
    assert st == L.LNOCC_OK, L.lnocc_status_string(st)
    assert abs(fs.e_mp2 - ref.e_mp2) < 1e-12
    assert abs(fs.e_ccsd - ref.e_ccsd) < 1e-8
    assert abs(fs.e_t - ref_t) < 1e-8
    np.testing.assert_allclose(host(t2), ref.t2, rtol=0, atol=1e-7)
    np.testing.assert_allclose(host(t1), ref.t1, rtol=0, atol=1e-7)
    assert fs.residual <= 1e-10


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-6), ("bf16", 5e-3)])
def test_mixed_precision_solve(precision, tol):
    """Ladder and (T) products in FP32 / BF16 (FP32 accumulation), everything
    else FP64: energies against the FP64 oracle.  FP32 keeps |dE| below the
    1e-6 Eh target; BF16 operands (8-bit mantissa) do not and are held to a
    looser bound that documents the size of the error."""
    say(f"mixed precision solve {precision}")
    o, v, X, seed = 6, 45, 100, 5
    f = make_fragment(o, v, X, seed)
    ref = occ.ccsd(f.B, f.eps_occ, f.eps_vir, conv_tol=1e-10)
    ref_t = otr.e_triples_restricted(f.B, f.eps_occ, f.eps_vir, ref.t1, ref.t2)
    B, eo, ev = _fragment_on_device(f)
    t1 = torch.empty((o, v), dtype=torch.float64, device=DEV)
    t2 = torch.empty((o, o, v, v), dtype=torch.float64, device=DEV)
    st, fs = _call(L.lnocc_fragment_ccsd, f, B, eo, ev, t1, t2, conv_tol=1e-9,
                   precision=precision)
    say(f"  {precision}: dE_ccsd={fs.e_ccsd - ref.e_ccsd:.3e} dE_t={fs.e_t - ref_t:.3e} "
        f"iters={fs.n_iter} status={st}")
    assert st in (L.LNOCC_OK, L.LNOCC_NOT_CONVERGED)
    assert abs(fs.e_ccsd - ref.e_ccsd) < tol * max(1.0, abs(ref.e_ccsd) * 10)
    assert abs(fs.e_t - ref_t) < tol


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-6), ("bf16", 5e-3)])
def test_mixed_precision_on_the_fly_ladder(precision, tol):
    """The ladder built in every iteration from the T1-dressed B_vv (converted
    to the low precision), written one block of a at a time (a chunk of a few
    a values, so several blocks and a short last one run) and contracted with
    split-bf16 (FP32) or bf16 products: energies against the FP64 oracle at
    the same bounds as the stored ladder."""
    say(f"mixed precision on-the-fly ladder {precision}")
    o, v, X, seed = 6, 45, 100, 5
    f = make_fragment(o, v, X, seed)
    ref = occ.ccsd(f.B, f.eps_occ, f.eps_vir, conv_tol=1e-10)
    ref_t = otr.e_triples_restricted(f.B, f.eps_occ, f.eps_vir, ref.t1, ref.t2)
    B, eo, ev = _fragment_on_device(f)
    t1 = torch.empty((o, v), dtype=torch.float64, device=DEV)
    t2 = torch.empty((o, o, v, v), dtype=torch.float64, device=DEV)
    st, fs = _call(L.lnocc_fragment_ccsd, f, B, eo, ev, t1, t2, conv_tol=1e-9,
                   precision=precision, ladder="on_the_fly", ladder_chunk_bytes=v ** 3 * 4 * 7)
    say(f"  {precision}: dE_ccsd={fs.e_ccsd - ref.e_ccsd:.3e} dE_t={fs.e_t - ref_t:.3e} "
        f"iters={fs.n_iter} status={st}")
    assert st in (L.LNOCC_OK, L.LNOCC_NOT_CONVERGED)
    assert abs(fs.e_ccsd - ref.e_ccsd) < tol * max(1.0, abs(ref.e_ccsd) * 10)
    assert abs(fs.e_t - ref_t) < tol


def _golden(name):
    import json
    import pathlib
    path = pathlib.Path(__file__).resolve().parent / "golden" / f"{name}.json"
    if not path.exists():
        pytest.skip(f"{path.name} not generated")
    return json.loads(path.read_text())


@pytest.mark.parametrize("precision,tol_e", [("fp64", 1e-8), ("fp32", 1e-6)])
def test_realistic_fragment_against_stored_oracle(precision, tol_e):
    """nocc=16, nvir=160, naux=528 (the benchmark workload, several tiles in
    every mode and a ragged 160 = 128 + 32 edge) against oracle values stored
    by tests/golden/make_golden.py."""
    g = _golden("single_realistic")
    say(f"realistic fragment {precision}")
    f = make_fragment(g["nocc"], g["nvir"], g["naux"], g["seed"])
    assert f.sha256() == g["input_sha256"]
    o, v = f.nocc, f.nvir
    B, eo, ev = _fragment_on_device(f)
    t1 = torch.empty((o, v), dtype=torch.float64, device=DEV)
    t2 = torch.empty((o, o, v, v), dtype=torch.float64, device=DEV)
    # FP32 ladder and (T) products leave a residual floor near 1e-9: converge to 1e-8
    tol = g["conv_tol"] if precision == "fp64" else 1e-8
    st, fs = _call(L.lnocc_fragment_ccsd, f, B, eo, ev, t1, t2, conv_tol=tol, precision=precision)
    say(f"  dE_mp2={fs.e_mp2 - g['e_mp2']:.2e} dE_ccsd={fs.e_ccsd - g['e_ccsd']:.2e} "
        f"dE_t={fs.e_t - g['e_t']:.2e} iters={fs.n_iter} (oracle {g['n_iter']})")
    assert st == L.LNOCC_OK
    assert abs(fs.e_mp2 - g["e_mp2"]) < 1e-10
    assert abs(fs.e_ccsd - g["e_ccsd"]) < tol_e
    assert abs(fs.e_t - g["e_t"]) < tol_e
    T2 = host(t2)
    idx = np.array(g["t2_index"])
    got = T2[idx[:, 0], idx[:, 1], idx[:, 2], idx[:, 3]]
    np.testing.assert_allclose(got, g["t2_value"], rtol=0, atol=1e-7 if precision == "fp64" else 1e-6)
    assert abs(np.linalg.norm(T2) - g["t2_norm"]) < 1e-7 * g["t2_norm"] * (1 if precision == "fp64" else 10)


def test_large_fragment_at_full_size():
    """The large workload (nocc=32, nvir=400, naux=1300: the ladder is formed on
    the fly, no v^4 storage) at full size.  The MP2 energy and a seeded sample of
    the MP1 amplitudes against oracle values stored by tests/golden/make_golden.py
    (large:mp2); the energy of that start (T1 = 0, so equal to E_MP2); and one full
    residual evaluation at those amplitudes, which must be finite and keep the
    pair symmetry R_ij^ab = R_ji^ba of the closed-shell equations."""
    g = _golden("large_mp2")
    say("large fragment at full size: MP2 start and one residual")
    f = make_fragment(g["nocc"], g["nvir"], g["naux"], g["seed"])
    assert f.sha256() == g["input_sha256"]
    o, v = f.nocc, f.nvir
    B, eo, ev = _fragment_on_device(f)
    del f
    t1 = torch.empty((o, v), dtype=torch.float64, device=DEV)
    t2 = torch.empty((o, o, v, v), dtype=torch.float64, device=DEV)
    st, fs = _call(L.lnocc_fragment_ccsd, None, B, eo, ev, t1, t2, max_iter=0,
                   do_triples=False)
    say(f"  dE_mp2={fs.e_mp2 - g['e_mp2']:.2e} ladder on the fly")
    assert st == L.LNOCC_OK
    assert abs(fs.e_mp2 - g["e_mp2"]) < 1e-10
    assert abs(fs.e_ccsd - fs.e_mp2) < 1e-12
    idx = np.array(g["t2_index"])
    got = host(t2[idx[:, 0], idx[:, 1], idx[:, 2], idx[:, 3]])
    np.testing.assert_allclose(got, g["t2_value"], rtol=0, atol=1e-13)
    assert abs(float(torch.linalg.vector_norm(t2)) - g["t2_norm"]) < 1e-12 * g["t2_norm"]
    assert float(t1.abs().max()) == 0.0
    r1 = torch.empty((o, v), dtype=torch.float64, device=DEV)
    r2 = torch.empty((o, o, v, v), dtype=torch.float64, device=DEV)
    opt = L.make_options()
    fr = L.make_fragment_struct(B, eo, ev, t1, t2, 1e-8)
    ws = L.Workspace(DEV)
    ws.attach([fr], opt)
    st = L.lnocc_ccsd_residuals(fr, opt, r1.data_ptr(), r2.data_ptr())
    assert st == L.LNOCC_OK, L.lnocc_last_error()
    assert bool(torch.isfinite(r1).all()) and bool(torch.isfinite(r2).all())
    scale = float(r2.abs().max())
    asym = float((r2 - r2.permute(1, 0, 3, 2)).abs().max())
    say(f"  |R2| max {scale:.3e}, pair asymmetry {asym:.1e}")
    assert scale > 0.0 and asym <= 1e-12 * scale
    del r2, t2, B, ws
    torch.cuda.empty_cache()


def test_solve_is_bitwise_reproducible():
    say("determinism o=4 v=20")
    f = make_fragment(4, 20, 72, 0)
    B, eo, ev = _fragment_on_device(f)
    out = []
    for _ in range(2):
        t1 = torch.empty((4, 20), dtype=torch.float64, device=DEV)
        t2 = torch.empty((4, 4, 20, 20), dtype=torch.float64, device=DEV)
        st, fs = _call(L.lnocc_fragment_ccsd, f, B, eo, ev, t1, t2)
        assert st == L.LNOCC_OK
        out.append((fs.e_ccsd, fs.e_t, fs.n_iter, host(t2).tobytes()))
    assert out[0] == out[1]


def test_error_paths_on_device():
    say("error paths")
    f = make_fragment(3, 8, 20, 4)
    B, eo, ev = _fragment_on_device(f)
    t1 = torch.empty((3, 8), dtype=torch.float64, device=DEV)
    t2 = torch.empty((3, 3, 8, 8), dtype=torch.float64, device=DEV)
    # overlapping spectrum: rejected before any solve
    bad = ev.clone()
    bad[0] = eo.max() + 0.0
    st, _ = _call(L.lnocc_fragment_ccsd, f, B, eo, bad, t1, t2)
    assert st == L.LNOCC_EINVAL
    # non-finite energy
    nan = eo.clone()
    nan[1] = float("nan")
    st, _ = _call(L.lnocc_fragment_ccsd, f, B, nan, ev, t1, t2)
    assert st == L.LNOCC_EINVAL
    # workspace too small
    opt = L.make_options()
    fs = L.make_fragment_struct(B, eo, ev, t1, t2, 1e-8)
    ws = L.Workspace(DEV)
    ws.attach([fs], opt)
    opt.workspace_bytes -= 4096
    assert L.lnocc_fragment_ccsd(fs, opt) == L.LNOCC_ENOMEM
    # iteration limit: warning, last iterate and its energy returned
    st, fs = _call(L.lnocc_fragment_ccsd, f, B, eo, ev, t1, t2, max_iter=1, do_triples=False)
    assert st == L.LNOCC_NOT_CONVERGED and fs.n_iter == 1 and np.isfinite(fs.e_ccsd)
    # no iteration: energy of the MP2 guess
    st, fs = _call(L.lnocc_fragment_ccsd, f, B, eo, ev, t1, t2, max_iter=0, do_triples=False)
    assert st == L.LNOCC_OK and fs.e_ccsd == fs.e_mp2


def test_restart_from_converged_amplitudes():
    say("restart")
    f = make_fragment(4, 20, 72, 0)
    B, eo, ev = _fragment_on_device(f)
    t1 = torch.empty((4, 20), dtype=torch.float64, device=DEV)
    t2 = torch.empty((4, 4, 20, 20), dtype=torch.float64, device=DEV)
    st, fs = _call(L.lnocc_fragment_ccsd, f, B, eo, ev, t1, t2, conv_tol=1e-10)
    assert st == L.LNOCC_OK
    st2, fs2 = _call(L.lnocc_fragment_ccsd, f, B, eo, ev, t1, t2, conv_tol=1e-9,
                     guess=L.LNOCC_GUESS_USER)
    assert st2 == L.LNOCC_OK and fs2.n_iter == 1
    assert abs(fs2.e_ccsd - fs.e_ccsd) < 1e-10 and abs(fs2.e_t - fs.e_t) < 1e-10


@pytest.mark.parametrize("o,v,X,seed,precision", [(4, 20, 72, 0, "fp64"), (6, 45, 100, 5, "fp32")])
def test_graph_replay_equals_eager(o, v, X, seed, precision):
    """The residual evaluation captured once as a HIP graph and replayed in
    every iteration (with the eager Jacobi / DIIS work between replays) gives
    bit-for-bit the eager solve."""
    say(f"graph replay o={o} v={v} {precision}")
    f = make_fragment(o, v, X, seed)
    B, eo, ev = _fragment_on_device(f)
    out = []
    for graphs in (False, True, True):
        t1 = torch.empty((o, v), dtype=torch.float64, device=DEV)
        t2 = torch.empty((o, o, v, v), dtype=torch.float64, device=DEV)
        st, fs = _call(L.lnocc_fragment_ccsd, f, B, eo, ev, t1, t2, conv_tol=1e-9,
                       precision=precision, graphs=graphs)
        assert st == L.LNOCC_OK
        out.append((fs.e_ccsd, fs.e_t, fs.n_iter, host(t2).tobytes()))
    assert out[0] == out[1] == out[2]


def test_autotuned_mixed_precision_solve():
    """Tuned plans in the FP32 mode (where the FP32-only tiles compete) keep the
    energies at FP32 rounding distance from the untuned solve."""
    say("autotune fp32")
    L.lnocc_autotune_clear()
    f = make_fragment(6, 45, 100, 5)
    B, eo, ev = _fragment_on_device(f)
    res = []
    for autotune in (False, True):
        t1 = torch.empty((6, 45), dtype=torch.float64, device=DEV)
        t2 = torch.empty((6, 6, 45, 45), dtype=torch.float64, device=DEV)
        st, fs = _call(L.lnocc_fragment_ccsd, f, B, eo, ev, t1, t2, conv_tol=1e-9,
                       precision="fp32", autotune=autotune)
        assert st == L.LNOCC_OK
        res.append((fs.e_ccsd, fs.e_t))
    L.lnocc_autotune_clear()
    assert abs(res[1][0] - res[0][0]) < 1e-8 and abs(res[1][1] - res[0][1]) < 1e-8


def test_autotuned_plans_keep_the_results(tmp_path):
    """Tile / split plans chosen by timing every candidate change only the
    summation order: energies agree with the heuristic choice to rounding, and
    the plans survive a save / clear / load round trip."""
    say("autotune")
    L.lnocc_autotune_clear()
    f = make_fragment(6, 45, 100, 5)
    B, eo, ev = _fragment_on_device(f)
    res = []
    for autotune in (False, True, True):
        t1 = torch.empty((6, 45), dtype=torch.float64, device=DEV)
        t2 = torch.empty((6, 6, 45, 45), dtype=torch.float64, device=DEV)
        st, fs = _call(L.lnocc_fragment_ccsd, f, B, eo, ev, t1, t2, conv_tol=1e-10,
                       autotune=autotune)
        assert st == L.LNOCC_OK
        res.append((fs.e_ccsd, fs.e_t, fs.n_iter))
    say(f"  heuristic {res[0]}, tuned {res[1]}, reused {res[2]}")
    assert abs(res[1][0] - res[0][0]) < 1e-10 and abs(res[1][1] - res[0][1]) < 1e-10
    # the setup contractions of the first tuned solve ran before any plan existed
    assert abs(res[2][0] - res[1][0]) < 1e-12 and abs(res[2][1] - res[1][1]) < 1e-12
    path = tmp_path / "plans.txt"
    n = L.lnocc_autotune_save(path)
    assert n > 10 and len(path.read_text().splitlines()) == n
    L.lnocc_autotune_clear()
    assert L.lnocc_autotune_load(path) == n
    L.lnocc_autotune_clear()
