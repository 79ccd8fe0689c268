"""Pins of the oracle's model of the precision arms (not in the paper): the
bfloat16 and OCP E4M3 quantizers, the per-row fp8 scale, the prefilter
ranking and the exact k-NN of the kept candidates.

Each quantity is checked against something the oracle does not compute:
torch's bfloat16 and float8_e4m3fn conversions (library routines), bit
arithmetic on float32 patterns, the closed-form E4M3 table, the special
cases where a quantizer is lossless (then the prefilter is the exact
distance and the arm reduces to the plain k-NN of S), and a brute-force
re-ranking from torch's quantizers on small inputs.
"""
import numpy as np
import pytest

import oracle
from paper_1509_06957_amd import workloads as W

torch = pytest.importorskip("torch")


# ----------------------------------------------------------------- E4M3 format

def _e4m3_closed_form(code):
    """OCP 8-bit float E4M3 ("FN"): bias 7, subnormals m/8 * 2^-6, S.1111.111 NaN."""
    s, e, m = code >> 7, (code >> 3) & 15, code & 7
    if e == 15 and m == 7:
        return np.nan
    mag = (m / 8.0) * 2.0 ** -6 if e == 0 else (1 + m / 8.0) * 2.0 ** (e - 7)
    return -mag if s else mag


def test_e4m3_decode_table_matches_torch_and_closed_form():
    codes = np.arange(256)
    got = oracle.e4m3_value(codes)
    ref = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).double().numpy()
    cf = np.array([_e4m3_closed_form(c) for c in codes])
    nan = np.isnan(got)
    assert nan.tolist() == np.isnan(ref).tolist() == np.isnan(cf).tolist()
    assert set(np.nonzero(nan)[0].tolist()) == {0x7F, 0xFF}
    assert np.array_equal(got[~nan], ref[~nan]) and np.array_equal(got[~nan], cf[~nan])
    assert got[0x7E] == 448.0 and got[0x01] == 2.0 ** -9 and got[0x38] == 1.0 and got[0x77] == 240.0
    assert np.signbit(got[0x80]) and got[0x80] == 0.0


def _finite_positive_values():
    v = oracle.e4m3_value(np.arange(0x7F))
    return v                      # ascending: 0 .. 448


def test_e4m3_rounding_midpoints_go_to_even():
    vals = _finite_positive_values()
    for c in range(len(vals) - 1):
        mid = np.float32((vals[c] + vals[c + 1]) / 2)
        assert float(mid) == (vals[c] + vals[c + 1]) / 2          # midpoints are float32-exact here
        want = c if c % 2 == 0 else c + 1
        assert int(oracle.e4m3_round(mid)) == want, f"midpoint of codes {c}, {c + 1}"
        assert int(oracle.e4m3_round(-mid)) == 0x80 | want
        below = np.nextafter(mid, np.float32(0))
        above = np.nextafter(mid, np.float32(np.inf))
        assert int(oracle.e4m3_round(below)) == c
        assert int(oracle.e4m3_round(above)) == c + 1


def test_e4m3_rounding_matches_torch():
    rng = np.random.default_rng(3)
    y = np.concatenate([rng.uniform(-240, 240, 20000), rng.uniform(-1, 1, 20000),
                        rng.uniform(-0.01, 0.01, 5000)]).astype(np.float32)
    vals = _finite_positive_values()
    mids = ((vals[:-1] + vals[1:]) / 2).astype(np.float32)
    y = np.concatenate([y, mids, -mids, np.nextafter(mids, np.float32(0))])
    ours = oracle.e4m3_round(y)
    ref = torch.from_numpy(y).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(ours, ref)


# ----------------------------------------------------------------- bfloat16

def _bf16_bits(x):
    """Round to nearest even by integer arithmetic on the float32 pattern."""
    b = x.view(np.uint32).astype(np.uint64)
    return ((b + 0x7FFF + ((b >> 16) & 1)) >> 16).astype(np.uint16)


def test_bf16_matches_bit_arithmetic_and_torch():
    rng = np.random.default_rng(5)
    pats = rng.integers(0, 2 ** 32, size=200000, dtype=np.uint64).astype(np.uint32)
    x = pats.view(np.float32)
    x = x[np.isfinite(x) & (np.abs(x) < 3.3e38)]
    # exact midpoints (low half 0x8000) with even and odd upper halves, and their neighbours
    mids = ((rng.integers(0, 2 ** 16, size=20000).astype(np.uint32) << 16) | 0x8000).view(np.float32)
    mids = mids[np.isfinite(mids) & (np.abs(mids) < 3.3e38)]
    x = np.concatenate([x, mids, np.nextafter(mids, np.float32(0)), np.float32([0.0, -0.0, 1.0, 255.0, 256.0])])
    ours = oracle.bf16_round(x)
    assert np.array_equal(ours, _bf16_bits(x))
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)
    # midpoint ties keep an even last bit
    tie = oracle.bf16_round(mids)
    assert np.all(tie & 1 == 0)


def test_bf16_value_is_upper_half():
    b = np.array([0x3F80, 0xC000, 0x4380, 0x0001, 0x7F7F], dtype=np.uint16)
    assert oracle.bf16_value(b).tolist() == [1.0, -2.0, 256.0, float(np.uint32(1 << 16).view(np.float32)),
                                             float(np.uint32(0x7F7F0000).view(np.float32))]


# ----------------------------------------------------------------- fp8 rows

def test_fp8_rows_scale_codes_norm():
    rng = np.random.default_rng(9)
    X = (rng.standard_normal((300, 64)) * rng.uniform(0.01, 100, (300, 1))).astype(np.float32)
    X[7] = 0.0
    codes, scale, norm = oracle.fp8_rows(X)
    mx = np.abs(X).max(1)
    want_scale = np.where(mx > 0, (mx / np.float32(240)).astype(np.float32), np.float32(1))
    assert np.array_equal(scale.view(np.uint32), want_scale.astype(np.float32).view(np.uint32))
    y = (X / scale[:, None]).astype(np.float32)                  # float32 division, as the arm defines
    ref = torch.from_numpy(y).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(codes, ref)
    dec = scale[:, None].astype(np.float64) * \
        torch.from_numpy(ref).view(torch.float8_e4m3fn).double().numpy()
    assert np.allclose(norm, (dec * dec).sum(1), rtol=1e-14, atol=0)
    assert np.all(np.abs(y) <= 240.0 * (1 + 2 ** -23))
    assert np.all(codes[7] == 0) and scale[7] == 1.0 and norm[7] == 0.0


def test_fp8_rows_lossless_on_the_grid():
    # rows whose largest magnitude is 240 (scale exactly 1) and whose values
    # lie on the E4M3 grid are reproduced exactly
    grid = _finite_positive_values()
    grid = grid[grid <= 240]
    rng = np.random.default_rng(11)
    X = (rng.choice(grid, size=(50, 32)) * rng.choice([-1, 1], size=(50, 32))).astype(np.float32)
    X[:, 0] = 240.0
    codes, scale, norm = oracle.fp8_rows(X)
    assert np.all(scale == 1.0)
    assert np.array_equal(oracle.e4m3_value(codes), X.astype(np.float64))
    assert np.array_equal(norm, (X.astype(np.float64) ** 2).sum(1))


# ----------------------------------------------------------------- prefilter arm

@pytest.fixture(scope="module")
def small_index():
    rng = np.random.default_rng(21)
    X = rng.standard_normal((3000, 32)).astype(np.float32)
    Q = rng.standard_normal((40, 32)).astype(np.float32)
    ix = oracle.build_index(X, 6, 4, 0.4, 7)
    return X, Q, ix


@pytest.mark.parametrize("arm", [oracle.ARM_BF16, oracle.ARM_FP8])
def test_prefilter_covering_s_is_the_plain_knn(small_index, arm):
    X, Q, ix = small_index
    plain = oracle.query(ix, Q, 10, 2, want_sets=True)
    kp = int(plain["s_count"].max())
    pf = oracle.query_prefilter(ix, Q, 10, 2, arm, kp)
    assert np.array_equal(pf["s_count"], plain["s_count"])
    assert np.array_equal(pf["idx"], plain["idx"]) and np.array_equal(pf["dist"], plain["dist"])
    assert np.array_equal(pf["keep_count"], plain["s_count"])
    for q in range(len(Q)):
        kept = pf["keep_ids"][q, :pf["keep_count"][q]]
        assert np.array_equal(np.sort(kept), plain["s_ids"][q])
        assert np.all(pf["keep_ids"][q, pf["keep_count"][q]:] == -1)


def test_bf16_prefilter_is_exact_on_8bit_integers():
    # integers <= 256 are exact in bfloat16: the score is the exact squared
    # distance, so the kept list is the exact top-kp of S and the answer the
    # plain k-NN of S
    rng = np.random.default_rng(23)
    X = rng.integers(0, 256, size=(4000, 24)).astype(np.float32)
    Q = rng.integers(0, 256, size=(30, 24)).astype(np.float32)
    ix = oracle.build_index(X, 5, 5, 0.5, 3)
    k, v, kp = 5, 1, 20
    plain = oracle.query(ix, Q, kp, v)
    pf = oracle.query_prefilter(ix, Q, k, v, oracle.ARM_BF16, kp)
    assert (pf["s_count"] > kp).all()
    assert np.array_equal(pf["keep_ids"], plain["idx"])
    sq = np.rint(plain["dist"] ** 2)                     # squared distances are integers here
    assert np.allclose(plain["dist"] ** 2, sq, rtol=1e-12, atol=0)
    assert np.array_equal(pf["keep_score"], sq)
    assert np.array_equal(pf["idx"], plain["idx"][:, :k])


def _rank_from_torch(X, Q, S, arm):
    """Brute-force prefilter ranking with torch's quantizers: squared float64
    distance to the decoded rows, order (score, id)."""
    Xs = X[S]
    if arm == oracle.ARM_BF16:
        dec = torch.from_numpy(Xs).to(torch.bfloat16).double().numpy()
    else:
        mx = np.abs(Xs).max(1)
        sc = np.where(mx > 0, (mx / np.float32(240)).astype(np.float32), np.float32(1))
        y = (Xs / sc[:, None]).astype(np.float32)
        dec = sc[:, None].astype(np.float64) * torch.from_numpy(y).to(torch.float8_e4m3fn).double().numpy()
    s = ((dec - Q.astype(np.float64)[None, :]) ** 2).sum(1)
    order = np.lexsort((S, s))
    return S[order], s[order]


@pytest.mark.parametrize("arm", [oracle.ARM_BF16, oracle.ARM_FP8])
def test_prefilter_ranking_brute_force(small_index, arm):
    X, Q, ix = small_index
    k, v, kp = 4, 1, 24
    plain = oracle.query(ix, Q, k, v, want_sets=True)
    pf = oracle.query_prefilter(ix, Q, k, v, arm, kp)
    for q in range(len(Q)):
        S = plain["s_ids"][q]
        ids, sc = _rank_from_torch(X, Q[q], S, arm)
        n = min(kp, len(S))
        assert np.array_equal(pf["keep_ids"][q, :n], ids[:n]), f"query {q}"
        assert np.allclose(pf["keep_score"][q, :n], sc[:n], rtol=1e-12, atol=0)
        kept = ids[:n]
        d = np.sqrt(((X[kept].astype(np.float64) - Q[q].astype(np.float64)) ** 2).sum(1))
        o = np.lexsort((kept, d))[:k]
        assert np.array_equal(pf["idx"][q, :min(k, n)], kept[o])
        assert np.allclose(pf["dist"][q, :min(k, n)], d[o], rtol=1e-14, atol=0)


def test_fp8_prefilter_lossy_on_gist_like_rows():
    # values in (0, 1) lose bits in E4M3: the kept list differs from the exact
    # top-kp for some queries, and the answer is still the k-NN of the kept
    w = W.GIST_LIKE.scaled(n=6000, nq=20, T=12, depth=2, v=2)
    X, Q = W.data(w), W.queries(w)
    ix = oracle.build_index(X, w.T, w.depth, w.a, w.index_seed)
    k, kp = 10, 40
    plain = oracle.query(ix, Q, kp, w.v)
    pf = oracle.query_prefilter(ix, Q, k, w.v, oracle.ARM_FP8, kp)
    assert (pf["s_count"] > kp).mean() > 0.5
    diff = [set(pf["keep_ids"][q].tolist()) != set(plain["idx"][q].tolist()) for q in range(len(Q))]
    assert any(diff)
    for q in range(len(Q)):
        kept = pf["keep_ids"][q, :pf["keep_count"][q]]
        d = np.sqrt(((X[kept].astype(np.float64) - Q[q].astype(np.float64)) ** 2).sum(1))
        o = np.lexsort((kept, d))[:k]
        m = len(o)
        assert np.array_equal(pf["idx"][q, :m], kept[o]) and np.all(pf["idx"][q, m:] == -1)
