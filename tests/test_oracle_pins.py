"""Pins for the FP64 oracle: it is checked against what the paper and the
mathematics fix, never against itself.

Each test names the passage it follows.  Kinds of pin used:
  * hand-worked examples (tests/golden/*.json, each with its citation);
  * brute force with explicit matrices and math.fsum on tiny inputs;
  * textbook identities (Kronecker form of the higher-order count sketch,
    vec(A X B) = (B^T kron A) vec(X));
  * exact moments over an exhaustive enumeration of the random hash draws
    (mean 0, variance ||p||^2/m, zero covariance, cross moment <u,v>/m);
  * closed forms of the collision probabilities (E2LSH p(R), SRP 1 - theta/pi)
    checked statistically;
  * library routines for special cases (NumPy matmul, torch's FP8/BF16 casts);
  * brute-force grouping and brute-force candidate scans for the index and
    the query, and the w -> infinity case where a query reduces to exact kNN.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _cs_matrix(h, s, m):
    """Explicit d x m count-sketch matrix S[j, h(j)] = s(j)."""
    d = len(h)
    S = np.zeros((d, m))
    S[np.arange(d), np.asarray(h)] = np.asarray(s, float)
    return S


def _fsum_matvec(x, S):
    return np.array([math.fsum(x[j] * S[j, l] for j in range(len(x))) for l in range(S.shape[1])])


# ---------------------------------------------------------------------------
# count sketch (Section 3.2, Definition def_cs, Eq. eq_cs)
# ---------------------------------------------------------------------------

def test_cs_worked_example(orc):
    g = _gold("cs_worked_example.json")
    y = orc.cs_sketch(np.array([g["x"]]), np.array(g["h"]), np.array(g["s"]), g["m"])
    assert y[0].tolist() == g["y"]


@pytest.mark.parametrize("d,m,seed", [(1, 1, 0), (7, 3, 1), (33, 8, 2), (64, 64, 3), (100, 128, 4)])
def test_cs_bruteforce_explicit_matrix(orc, d, m, seed):
    g = np.random.default_rng(seed)
    x = g.standard_normal((3, d))
    h = g.integers(0, m, d)
    s = g.choice([-1, 1], d)
    y = orc.cs_sketch(x, h, s, m)
    S = _cs_matrix(h, s, m)
    for i in range(3):
        np.testing.assert_allclose(y[i], _fsum_matvec(x[i], S), rtol=0, atol=1e-12)


def test_cs_special_hashes(orc):
    # all coordinates in one bin: the signed sum; identity hash (d = m): s * x
    g = np.random.default_rng(5)
    x = g.integers(-9, 10, (2, 6)).astype(float)
    s = g.choice([-1, 1], 6)
    y = orc.cs_sketch(x, np.zeros(6, np.uint32), s, 3)
    assert (y[:, 0] == (x * s).sum(1)).all() and (y[:, 1:] == 0).all()
    y = orc.cs_sketch(x, np.arange(6), s, 6)
    assert (y == x * s).all()


def test_cs_linearity_exact(orc):
    # CS(a x + b z) = a CS(x) + b CS(z); exact for small integers and dyadic a, b
    g = np.random.default_rng(6)
    x = g.integers(-50, 50, (4, 40)).astype(float)
    z = g.integers(-50, 50, (4, 40)).astype(float)
    h = g.integers(0, 9, 40)
    s = g.choice([-1, 1], 40)
    a, b = 0.75, -2.5
    lhs = orc.cs_sketch(a * x + b * z, h, s, 9)
    rhs = a * orc.cs_sketch(x, h, s, 9) + b * orc.cs_sketch(z, h, s, 9)
    assert (lhs == rhs).all()


def test_cs_exact_moments_enumeration(orc):
    """Over all h in [m]^d, s in {+-1}^d (uniform): E[CS_l] = 0, E[CS_l^2] = ||x||^2/m,
    E[CS_l CS_l'] = 0 (l != l'), E[CS(u)_l CS(v)_l] = <u,v>/m.
    Theorem uni_cs (mean and variance of each bin), Theorem mul_cs_new
    (covariance), Theorem cs_bi_variate (cross moment)."""
    d, m = 4, 3
    u = np.array([[3.0, -1.0, 2.0, 5.0]])
    v = np.array([[1.0, 4.0, -2.0, 1.0]])
    acc = {"mean": np.zeros(m), "sq": np.zeros(m), "cov01": 0.0, "cross": np.zeros(m)}
    cnt = 0
    for h in itertools.product(range(m), repeat=d):
        for s in itertools.product((-1, 1), repeat=d):
            yu = orc.cs_sketch(u, np.array(h), np.array(s), m)[0]
            yv = orc.cs_sketch(v, np.array(h), np.array(s), m)[0]
            acc["mean"] += yu
            acc["sq"] += yu * yu
            acc["cov01"] += yu[0] * yu[1]
            acc["cross"] += yu * yv
            cnt += 1
    assert cnt == m ** d * 2 ** d
    np.testing.assert_allclose(acc["mean"] / cnt, 0.0, atol=1e-12)
    np.testing.assert_allclose(acc["sq"] / cnt, (u * u).sum() / m, rtol=1e-12)
    assert abs(acc["cov01"] / cnt) < 1e-12
    np.testing.assert_allclose(acc["cross"] / cnt, (u * v).sum() / m, rtol=1e-12)


# ---------------------------------------------------------------------------
# higher-order count sketch (Section 3.2, Definition def_hcs, Eq. eqhcs)
# ---------------------------------------------------------------------------

def _mode_matrix(hk, sk, mk):
    """C_k[l, i] = s_k(i) [h_k(i) = l]  (m_k x d_k)."""
    Cm = np.zeros((mk, len(hk)))
    Cm[np.asarray(hk), np.arange(len(hk))] = np.asarray(sk, float)
    return Cm


def _hcs_state(dk, mk, seed):
    g = np.random.default_rng(seed)
    hk = [g.integers(0, mm, dd) for dd, mm in zip(dk, mk)]
    sk = [g.choice([-1, 1], dd) for dd in dk]
    return hk, sk


@pytest.mark.parametrize("dk,mk", [((4,), (3,)), ((4, 5), (2, 3)), ((3, 4, 2), (2, 2, 3)),
                                   ((8, 8), (4, 4)), ((2, 3, 2, 2), (2, 1, 2, 2))])
def test_hcs_kronecker_identity(orc, dk, mk):
    """vec(HCS(p)) = (C_N kron ... kron C_1) vec(p) with vec = first mode fastest."""
    hk, sk = _hcs_state(dk, mk, 11)
    D = int(np.prod(dk))
    x = np.random.default_rng(12).standard_normal((2, D))
    y = orc.hcs_sketch(x, dk, mk, hk, sk)
    M = np.ones((1, 1))
    for k in range(len(dk)):
        M = np.kron(_mode_matrix(hk[k], sk[k], mk[k]), M)
    np.testing.assert_allclose(y, x @ M.T, rtol=0, atol=1e-12)


def test_hcs_order2_matrix_form(orc):
    """N = 2: HCS(P) = C_1 P C_2^T for P = reshape(p, d_1 x d_2) first mode fastest (Section 1)."""
    dk, mk = (6, 5), (3, 4)
    hk, sk = _hcs_state(dk, mk, 13)
    p = np.random.default_rng(14).standard_normal(30)
    P = p.reshape(dk, order="F")
    C1, C2 = _mode_matrix(hk[0], sk[0], mk[0]), _mode_matrix(hk[1], sk[1], mk[1])
    want = (C1 @ P @ C2.T).reshape(-1, order="F")
    np.testing.assert_allclose(orc.hcs_sketch(p[None], dk, mk, hk, sk)[0], want, atol=1e-12)


def test_hcs_order1_is_cs(orc):
    g = np.random.default_rng(15)
    x = g.standard_normal((3, 20))
    h = g.integers(0, 7, 20)
    s = g.choice([-1, 1], 20)
    assert (orc.hcs_sketch(x, (20,), (7,), [h], [s]) == orc.cs_sketch(x, h, s, 7)).all()


def test_hcs_is_cs_under_composite_hash(orc):
    """bin(j) = sum_k h_k(i_k) prod_{t<k} m_t, sign(j) = prod_k s_k(i_k) (Definition def_hcs)."""
    dk, mk = (4, 3, 5), (2, 3, 2)
    hk, sk = _hcs_state(dk, mk, 16)
    D = 60
    hb, sb = np.zeros(D, int), np.zeros(D, int)
    for j in range(D):
        i1, i2, i3 = j % 4, (j // 4) % 3, j // 12
        hb[j] = hk[0][i1] + mk[0] * (hk[1][i2] + mk[1] * hk[2][i3])
        sb[j] = sk[0][i1] * sk[1][i2] * sk[2][i3]
    x = np.random.default_rng(17).integers(-20, 20, (3, D)).astype(float)
    assert (orc.hcs_sketch(x, dk, mk, hk, sk) == orc.cs_sketch(x, hb, sb, 12)).all()


def test_hcs_zero_padding(orc):
    """d not a product of the mode sizes: pad with zeros at the end (Section 6)."""
    dk, mk = (4, 4), (2, 2)
    hk, sk = _hcs_state(dk, mk, 18)
    x = np.random.default_rng(19).standard_normal((2, 13))
    xp = np.concatenate([x, np.zeros((2, 3))], 1)
    assert (orc.hcs_sketch(x, dk, mk, hk, sk) == orc.hcs_sketch(xp, dk, mk, hk, sk)).all()


def test_hcs_exact_moments_enumeration(orc):
    """Theorem hcs_normality: mean 0, variance ||p||^2/m for each bin; Theorem
    hcs_normality_multi: zero covariance between bins.  Exhaustive over all
    per-mode hashes and signs for d = 2 x 2, m = 2 x 2."""
    dk, mk = (2, 2), (2, 2)
    x = np.array([[1.0, -3.0, 2.0, 4.0]])
    m = 4
    tot, sq, cov, cnt = np.zeros(m), np.zeros(m), np.zeros((m, m)), 0
    for h1 in itertools.product(range(2), repeat=2):
        for h2 in itertools.product(range(2), repeat=2):
            for s1 in itertools.product((-1, 1), repeat=2):
                for s2 in itertools.product((-1, 1), repeat=2):
                    y = orc.hcs_sketch(x, dk, mk, [np.array(h1), np.array(h2)],
                                       [np.array(s1), np.array(s2)])[0]
                    tot += y
                    sq += y * y
                    cov += np.outer(y, y)
                    cnt += 1
    np.testing.assert_allclose(tot / cnt, 0, atol=1e-12)
    np.testing.assert_allclose(sq / cnt, (x * x).sum() / m, rtol=1e-12)
    off = cov / cnt - np.diag(np.diag(cov / cnt))
    np.testing.assert_allclose(off, 0, atol=1e-12)


# ---------------------------------------------------------------------------
# assignment of sketch components to tables (reading of which components form
# a table; the paper leaves it open)
# ---------------------------------------------------------------------------

def test_assign_components_permutation_matrix(orc):
    """Position slot[l] receives component l: y' = y P with P[l, slot[l]] = 1,
    and the identity map leaves y unchanged; hand case m = 4."""
    y = np.array([[10.0, 20.0, 30.0, 40.0]])
    out = orc.assign_components(y, np.array([2, 0, 3, 1]))
    assert out.tolist() == [[20.0, 40.0, 10.0, 30.0]]
    g = np.random.default_rng(23)
    m = 48
    y = g.standard_normal((5, m))
    slot = g.permutation(m)
    P = np.zeros((m, m))
    P[np.arange(m), slot] = 1.0
    assert (orc.assign_components(y, slot) == y @ P).all()
    assert (orc.assign_components(y, np.arange(m)) == y).all()


def test_hcs_with_slots_is_cs_under_composite_slot_hash(orc):
    """HCS followed by the component map equals a count sketch whose bin of
    coordinate j is slot[composite bin(j)] (Definition def_hcs)."""
    dk, mk = (4, 3, 5), (2, 3, 2)
    hk, sk = _hcs_state(dk, mk, 24)
    slot = np.random.default_rng(25).permutation(12)
    hb, sb = np.zeros(60, int), np.zeros(60, int)
    for j in range(60):
        i1, i2, i3 = j % 4, (j // 4) % 3, j // 12
        hb[j] = slot[hk[0][i1] + mk[0] * (hk[1][i2] + mk[1] * hk[2][i3])]
        sb[j] = sk[0][i1] * sk[1][i2] * sk[2][i3]
    x = np.random.default_rng(26).integers(-20, 20, (3, 60)).astype(float)
    b = np.zeros(12, np.float32)
    a = orc.hash_points(x, orc.SRP, 3, 4, kind="hcs", dk=dk, mk=mk, hk=hk, sk=sk,
                        comp_slot=slot)
    c = orc.hash_points(x, orc.SRP, 3, 4, kind="cs", h=hb, s=sb)
    assert (a["y"] == c["y"]).all() and (a["keys"] == c["keys"]).all()
    e = orc.hash_points(x, orc.E2LSH, 3, 4, kind="hcs", dk=dk, mk=mk, hk=hk, sk=sk, w=2.0, b=b,
                        comp_slot=slot)
    f = orc.hash_points(x, orc.E2LSH, 3, 4, kind="cs", h=hb, s=sb, w=2.0, b=b)
    assert (e["codes"] == f["codes"]).all() and (e["keys"] == f["keys"]).all()


def _structurally_zero_tables(dk, mk, hk, K, slot):
    """Tables all of whose code positions hold a sketch component that no
    input index reaches (some mode bin l_k with no i_k mapped to it)."""
    hit = [np.bincount(h, minlength=m) > 0 for h, m in zip(hk, mk)]
    live = hit[0]
    for k in range(1, len(dk)):
        live = np.concatenate([live & hk_live for hk_live in hit[k]])   # l = l_1 + m_1 l_2 + ...
    pos_live = np.zeros(live.size, bool)
    pos_live[slot] = live
    return int((~pos_live.reshape(-1, K).any(axis=1)).sum())


def test_c3_tables_not_constant_with_slots():
    """The 500k x 4096 tensor-reshape workload, K = 16, L = 64: with contiguous
    tables some tables sit inside one empty mode bin (every point gets the same
    code there); with the workload's seeded component map none does."""
    from paper_2503_06737_amd import synth
    wl = synth.C3
    slot = wl.slots()
    for i in range(len(wl.hcs)):
        dk, mk = wl.hcs[i]
        hk, _ = wl.hcs_state(i)
        assert _structurally_zero_tables(dk, mk, hk, wl.K, np.arange(wl.m)) > 0
        assert _structurally_zero_tables(dk, mk, hk, wl.K, slot) == 0


# ---------------------------------------------------------------------------
# dense projection (Section 3.1, Definitions e2lsh and srp)
# ---------------------------------------------------------------------------

def test_dense_matches_matmul(orc):
    g = np.random.default_rng(20)
    x = g.standard_normal((5, 37))
    R = g.standard_normal((37, 11)).astype(np.float32)
    np.testing.assert_allclose(orc.dense_proj(x, R), x @ R.astype(np.float64), rtol=1e-12,
                               atol=1e-12)


def test_dense_with_cs_matrix_is_cs(orc):
    """Dense projection by the explicit count-sketch matrix equals the count sketch."""
    g = np.random.default_rng(21)
    x = g.integers(-30, 30, (4, 25)).astype(float)
    h, s = g.integers(0, 6, 25), g.choice([-1, 1], 25)
    R = _cs_matrix(h, s, 6).astype(np.float32)
    assert (orc.dense_proj(x, R) == orc.cs_sketch(x, h, s, 6)).all()


# ---------------------------------------------------------------------------
# discretisation
# ---------------------------------------------------------------------------

def test_discretise_hand_cases(orc):
    g = _gold("discretise_cases.json")
    y = np.array(g["y"])
    b = np.array(g["b"], np.float32)
    codes, near = orc.disc_e2lsh(y, b, g["w"], math.sqrt(g["m"]))
    assert codes.tolist() == g["codes_sqrt_m"]
    assert near.tolist() == g["near_edge_sqrt_m"]
    codes, _ = orc.disc_e2lsh(y, b, g["w"], 1.0)
    assert codes.tolist() == g["codes_dense"]
    bits, _ = orc.disc_srp(y, np.ones(2))
    assert bits.tolist() == g["srp_bits"]


def test_srp_near_edge_band_uses_row_norm(orc):
    """The SRP near-edge band is |y| < 1e-6 * ||x||_2, with ||x||_2 of the row
    being hashed (worked cases: rows (3, 4, t), band 5e-6).  A band built from
    ||x||^2, max|x| or ||x||_1 fails one of the rows."""
    g = _gold("srp_near_edge_cases.json")
    x = np.array(g["x"])
    out = orc.hash_points(x, orc.SRP, 1, g["m"], kind="cs", h=np.array(g["h"]),
                          s=np.array(g["s"]))
    assert out["codes"].tolist() == g["bits"]
    assert out["near"].tolist() == g["near"]
    # the same band through disc_srp with the norms passed explicitly
    bits, near = orc.disc_srp(x, np.full(len(x), 5.0))
    assert near.tolist() == g["near"] and bits.tolist() == g["bits"]


def test_row_norms_pythagorean(orc):
    g = _gold("row_norm_cases.json")
    assert orc.row_norms(np.array(g["rows"])).tolist() == g["norms"]


def test_e2lsh_codes_saturate_to_int32(orc):
    """floor(v / w) outside the int32 range saturates to its nearest end; the
    largest and smallest representable codes are kept exactly."""
    g = _gold("e2lsh_int32_saturation.json")
    for row in g["rows"]:
        y = np.array([row["y"]])
        codes, _ = orc.disc_e2lsh(y, np.zeros(y.shape[1], np.float32), row["w"], row["alpha"])
        assert codes[0].tolist() == row["codes"]


def test_hash_points_cs_e2lsh_uses_sqrt_m(orc):
    """CS-E2LSH scales the sketch by sqrt(m) before the shift (Definition CS_Eucl_LSH)."""
    g = np.random.default_rng(22)
    x = g.standard_normal((50, 64))
    h, s = g.integers(0, 16, 64), g.choice([-1, 1], 64)
    b = (g.random(16) * 2.0).astype(np.float32)
    out = orc.hash_points(x, orc.E2LSH, 4, 4, kind="cs", w=2.0, b=b, h=h, s=s)
    S = _cs_matrix(h, s, 16)
    v = 4.0 * (x @ S) + b.astype(float)
    want = np.floor(v / 2.0)
    ok = ~out["near"]
    assert (out["codes"][ok] == want[ok]).all()


# ---------------------------------------------------------------------------
# collision probabilities (Section 3.1 E2LSH p(R), Eq. eq191022 for SRP)
# ---------------------------------------------------------------------------

def _p_e2lsh_closed(c, w):
    r = w / c
    return 1 - 2 * stats.norm.cdf(-r) - 2 / (math.sqrt(2 * math.pi) * r) * (1 - math.exp(-r * r / 2))


def _p_e2lsh_integral(c, w):
    f = lambda t: 2 * stats.norm.pdf(t)          # density of |N(0,1)|
    return integrate.quad(lambda t: (1 / c) * f(t / c) * (1 - t / w), 0, w)[0]


@pytest.mark.parametrize("c", [0.5, 1.0, 2.5, 4.0, 9.0])
def test_e2lsh_closed_form_matches_paper_integral(c):
    assert abs(_p_e2lsh_closed(c, 4.0) - _p_e2lsh_integral(c, 4.0)) < 1e-9


@pytest.mark.parametrize("dist", [1.0, 3.0, 6.0])
def test_dense_e2lsh_collision_rate(orc, dist):
    """Dense E2LSH: Pr[h(p) = h(q)] = p(R) exactly, R = ||p - q|| (Section 3.1)."""
    g = np.random.default_rng(int(dist * 10))
    d, m, w = 12, 40000, 4.0
    p = g.standard_normal(d)
    u = g.standard_normal(d)
    q = p + dist * u / np.linalg.norm(u)
    R = g.standard_normal((d, m)).astype(np.float32)
    b = (g.random(m) * w).astype(np.float32)
    Rm = R.astype(np.float64)
    # exact distance under the float32 matrix is the same vector norm
    y = orc.dense_proj(np.stack([p, q]), R)
    codes, _ = orc.disc_e2lsh(y, b, w, 1.0)
    rate = (codes[0] == codes[1]).mean()
    pr = _p_e2lsh_closed(dist, w)
    assert abs(rate - pr) < 4.5 * math.sqrt(pr * (1 - pr) / m) + 1e-3
    assert Rm.shape == (d, m)


def test_e2lsh_shift_collision_given_projection(orc):
    """For a fixed projection gap delta, over b ~ U[0,w): Pr = max(0, 1 - |delta|/w)."""
    g = np.random.default_rng(30)
    w, m = 4.0, 60000
    b = (g.random(m) * w).astype(np.float32)
    for delta in (0.0, 0.5, 1.7, 3.9, 5.0):
        y = np.stack([np.full(m, 0.3), np.full(m, 0.3 + delta)])
        c, _ = orc.disc_e2lsh(y, b, w, 1.0)
        rate = (c[0] == c[1]).mean()
        want = max(0.0, 1 - abs(delta) / w)
        assert abs(rate - want) < 4.5 * math.sqrt(max(want * (1 - want), 1e-9) / m) + 1e-3


@pytest.mark.parametrize("cos", [0.9, 0.3, -0.5])
def test_dense_srp_collision_rate(orc, cos):
    """SRP: Pr[sgn<r,u> = sgn<r,v>] = 1 - theta/pi (Eq. eq191022)."""
    g = np.random.default_rng(40)
    d, m = 10, 40000
    u = g.standard_normal(d)
    u /= np.linalg.norm(u)
    z = g.standard_normal(d)
    z -= z.dot(u) * u
    z /= np.linalg.norm(z)
    v = cos * u + math.sqrt(1 - cos * cos) * z
    R = g.standard_normal((d, m)).astype(np.float32)
    y = orc.dense_proj(np.stack([u, v]), R)
    bits, _ = orc.disc_srp(y, np.ones(2))
    rate = (bits[0] == bits[1]).mean()
    want = 1 - math.acos(cos) / math.pi
    assert abs(rate - want) < 4.5 * math.sqrt(want * (1 - want) / m)


def test_cs_srp_collision_enumeration_tiny(orc):
    """CS-SRP on tiny d: the exact collision probability over all (h, s), by
    brute force with explicit matrices, equals the oracle's average; includes
    the sgn(0) = 0 convention (Definition cs_consine_lsh)."""
    d, m = 4, 2
    u = np.array([[1.0, 2.0, -1.0, 0.0]])
    v = np.array([[1.0, 1.0, 1.0, -2.0]])
    hits_o, hits_b, cnt = 0, 0, 0
    for h in itertools.product(range(m), repeat=d):
        for s in itertools.product((-1, 1), repeat=d):
            h_, s_ = np.array(h), np.array(s)
            bu, _ = orc.disc_srp(orc.cs_sketch(u, h_, s_, m), np.ones(1))
            bv, _ = orc.disc_srp(orc.cs_sketch(v, h_, s_, m), np.ones(1))
            hits_o += int(bu[0, 0] == bv[0, 0])
            S = _cs_matrix(h, s, m)
            yu, yv = u[0] @ S, v[0] @ S
            hits_b += int((yu[0] > 0) == (yv[0] > 0))
            cnt += 1
    assert hits_o == hits_b and cnt == 256


def test_cs_e2lsh_collision_large_d(orc):
    """CS-E2LSH collision rate approaches p(R) when d >> m (Theorem
    CS_Eucl_LSH_property; asymptotic, so a loose band)."""
    g = np.random.default_rng(50)
    d, m, w, trials = 4096, 8, 4.0, 1500
    p = g.standard_normal(d)
    u = g.standard_normal(d)
    q = p + 2.0 * u / np.linalg.norm(u)
    hits = 0
    for t in range(trials):
        h = g.integers(0, m, d)
        s = g.choice([-1, 1], d)
        b = (g.random(m) * w).astype(np.float32)
        out = orc.hash_points(np.stack([p, q]), orc.E2LSH, m, 1, kind="cs", w=w, b=b, h=h, s=s)
        hits += (out["codes"][0] == out["codes"][1]).sum()
    rate = hits / (trials * m)
    assert abs(rate - _p_e2lsh_closed(2.0, w)) < 0.02


# ---------------------------------------------------------------------------
# keys (Section 3.1: concatenation of K codes into the bucket of table t)
# ---------------------------------------------------------------------------

def test_mix64_published_vectors(orc):
    g = _gold("splitmix64_vectors.json")
    gamma = int(g["gamma"], 16)
    state = 0
    for want in g["outputs_seed0"]:
        state = (state + gamma) & 0xFFFFFFFFFFFFFFFF
        assert orc.mix64(state) == int(want, 16)


def test_srp_key_bit_order(orc):
    bits = np.array([[1, 0, 1, 1, 0, 0, 0, 1]], np.int32)   # K = 4, L = 2
    keys = orc.keys_srp(bits, 4, 2)
    assert keys[:, 0].tolist() == [0b1101, 0b1000]


def test_e2lsh_keys_equal_iff_tuples_equal(orc):
    g = np.random.default_rng(60)
    n, K, L = 20000, 16, 2
    codes = g.integers(-6, 7, (n, K * L)).astype(np.int32)
    codes[1::2] = codes[0::2]                     # every odd row duplicates its even neighbour
    codes[2, 5] = 200                             # one wide tuple in table 0
    codes[4, K + 3] = -129                        # one wide tuple in table 1
    keys = orc.keys_e2lsh(codes, K, L)
    for t in range(L):
        tup = {}
        for i in range(n):
            tup.setdefault(codes[i, t * K:(t + 1) * K].tobytes(), set()).add(int(keys[t, i]))
        assert all(len(v) == 1 for v in tup.values())           # equal tuples -> one key
        assert len({next(iter(v)) for v in tup.values()}) == len(tup)   # distinct -> distinct
    # the table index enters the key
    same = np.concatenate([codes[:, :K], codes[:, :K]], 1)
    k2 = orc.keys_e2lsh(same, K, 2)
    assert (k2[0] != k2[1]).all()


def test_e2lsh_key_sensitive_to_every_position_and_boundary(orc):
    K = 16
    base = np.zeros((1, K), np.int32)
    k0 = int(orc.keys_e2lsh(base, K, 1)[0, 0])
    seen = {k0}
    for r in range(K):
        for v in (-128, -1, 1, 127, 128, -129, 1 << 20):
            c = base.copy()
            c[0, r] = v
            k = int(orc.keys_e2lsh(c, K, 1)[0, 0])
            assert k not in seen
            seen.add(k)


# ---------------------------------------------------------------------------
# index (Section 3.1): each point in the bucket of its key, per table
# ---------------------------------------------------------------------------

def test_index_bruteforce_groupby(orc):
    g = np.random.default_rng(70)
    L, n, base = 3, 3000, 1000
    keys = g.integers(0, 50, (L, n)).astype(np.uint64) * np.uint64(0x9E3779B97F4A7C15)
    keys[1] = np.uint64(7)                          # one table with a single bucket
    keys[2, :5] = np.uint64(0xFFFFFFFFFFFFFFFF)     # extreme key values
    idx = orc.build_index(keys, id_base=base)
    for t in range(L):
        groups = {}
        for i in range(n):
            groups.setdefault(int(keys[t, i]), []).append(base + i)
        u = int(idx["nuniq"][t])
        assert u == len(groups)
        uk = idx["ukeys"][t, :u].tolist()
        assert uk == sorted(groups)
        o = idx["offs"][t]
        for j, kk in enumerate(uk):
            assert idx["sorted_ids"][t, o[j]:o[j + 1]].tolist() == groups[kk]
        assert o[u] == n
        assert sorted(idx["sorted_ids"][t].tolist()) == list(range(base, base + n))


def test_index_empty(orc):
    idx = orc.build_index(np.zeros((2, 0), np.uint64))
    assert idx["nuniq"].tolist() == [0, 0] and idx["offs"][:, 0].tolist() == [0, 0]


# ---------------------------------------------------------------------------
# query: union of the probed buckets, exact re-rank (Sections 3.1 and 6)
# ---------------------------------------------------------------------------

def _bruteforce_query(keys_list, base, q, qk, k, watermark, metric):
    cand = set()
    for keys, id0 in keys_list:
        L, n = keys.shape
        for t in range(L):
            for i in range(n):
                if keys[t, i] == qk[t] and id0 + i < watermark:
                    cand.add(id0 + i)
    sc = []
    for c in sorted(cand):
        x = base[c]
        if metric == 0:
            s = math.sqrt(math.fsum((q - x) ** 2))
        else:
            nq, nx = math.sqrt(math.fsum(q * q)), math.sqrt(math.fsum(x * x))
            s = 1 - (math.fsum(q * x) / (nq * nx) if nq > 0 and nx > 0 else 0.0)
        sc.append((s, c))
    sc.sort()
    return sc[:k], len(cand)


@pytest.mark.parametrize("metric", [0, 1])
def test_query_bruteforce(orc, metric):
    g = np.random.default_rng(80 + metric)
    d, L, k = 6, 4, 5
    base = g.standard_normal((400, d))
    base[17] = 0.0                                  # a zero vector (cos defined as 0)
    keys_a = g.integers(0, 6, (L, 250)).astype(np.uint64)
    keys_b = g.integers(0, 6, (L, 150)).astype(np.uint64)
    segs = [orc.build_index(keys_a, 0), orc.build_index(keys_b, 250)]
    Q = g.standard_normal((7, d))
    qk = g.integers(0, 7, (L, 7)).astype(np.uint64)
    for wm in (400, 300):
        ids, sc, nc = orc.query(segs, base, Q, qk, k, wm, metric)
        for i in range(7):
            want, ncand = _bruteforce_query([(keys_a, 0), (keys_b, 250)], base, Q[i], qk[:, i],
                                            k, wm, metric)
            assert nc[i] == ncand
            assert ids[i, :len(want)].tolist() == [c for _, c in want]
            np.testing.assert_allclose(sc[i, :len(want)], [s for s, _ in want], rtol=1e-12)
            assert (ids[i, len(want):] == -1).all() and np.isinf(sc[i, len(want):]).all()


def test_query_w_infinite_is_exact_knn(orc):
    """With w -> infinity and b drawn inside (0, w) every E2LSH code is 0, all
    points share one bucket per table, and the query returns the exact k
    nearest neighbours (b = w/2 here)."""
    g = np.random.default_rng(90)
    n, d, K, L, k = 500, 16, 4, 3, 10
    x = g.standard_normal((n, d))
    h, s = g.integers(0, K * L, d), g.choice([-1, 1], d)
    b = np.full(K * L, 0.5e30, np.float32)
    out = orc.hash_points(x, orc.E2LSH, K, L, kind="cs", w=1e30, b=b, h=h, s=s)
    idx = orc.build_index(out["keys"])
    assert (idx["nuniq"] == 1).all()
    Q = g.standard_normal((5, d))
    qo = orc.hash_points(Q, orc.E2LSH, K, L, kind="cs", w=1e30, b=b, h=h, s=s)
    ids, sc, nc = orc.query([idx], x, Q, qo["keys"], k, n, 0)
    for i in range(5):
        dist = np.sqrt(((x - Q[i]) ** 2).sum(1))
        order = np.lexsort((np.arange(n), dist))[:k]
        assert ids[i].tolist() == order.tolist()
        assert nc[i] == n


# ---------------------------------------------------------------------------
# decoding of stored values
# ---------------------------------------------------------------------------

def test_fp8_decode_matches_library_cast(orc):
    import torch
    allbits = torch.arange(256, dtype=torch.int32).to(torch.uint8)
    ref = allbits.view(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = np.array([orc.fp8_value(i) for i in range(256)])
    nan = np.isnan(ref)
    assert (np.isnan(got) == nan).all()
    assert (got[~nan] == ref[~nan]).all()


def test_bf16_and_scale_decode(orc):
    import torch
    g = np.random.default_rng(91)
    v = torch.from_numpy(g.standard_normal((4, 9)).astype(np.float32)).to(torch.bfloat16)
    bits = v.view(torch.int16).numpy().view(np.uint16)
    sc = np.array([1.0, 0.5, 3.25, 1e-3], np.float32)
    x = orc.decode(bits, sc)
    want = v.to(torch.float64).numpy() * sc.astype(np.float64)[:, None]
    assert (x == want).all()


# ---------------------------------------------------------------------------
# low-precision storage (quantisation)
# ---------------------------------------------------------------------------

def _quant_edge_rows():
    """Rows whose scale is 1 (max |x| = 1 for BF16, 448 for FP8) so their
    quotients are the values themselves: exact halfway cases, values that
    round to zero, signed zeros, the clamp, and a zero row."""
    bf = np.zeros((3, 12), np.float32)
    # BF16 steps are 2^-8 in [0.5, 1) and 2^-9 in [0.25, 0.5): 0.5 + 2^-9 is
    # halfway between 0.5 and 0.5 + 2^-8 (ties to even: 0.5), 0.5 + 3*2^-9
    # halfway between 0.5 + 2^-8 and 0.5 + 2^-7 (even: 0.5 + 2^-7),
    # 0.25 + 2^-10 halfway between 0.25 and 0.25 + 2^-9 (even: 0.25)
    bf[0, :8] = [1.0, 0.5 + 2 ** -9, 0.5 + 3 * 2 ** -9, -(0.5 + 2 ** -9), 0.25 + 2 ** -10, -0.0,
                 2 ** -140, 0.75]
    bf[1, :4] = [-1.0, 0.1, -0.3, 1e-30]
    # bf[2] is a zero row: scale 1, every code zero
    f8 = np.zeros((3, 12), np.float32)
    # E4M3FN near 1: step 1/8; 1 + 1/16 is halfway (even: 1.0), 1 + 3/16 (even: 1.25);
    # subnormal grid 2^-9: 2^-10 halfway between 0 and 2^-9 (even: 0), 3 * 2^-10 (even: 2^-8)
    f8[0, :10] = [448.0, 1 + 1 / 16, 1 + 3 / 16, -(1 + 1 / 16), 2 ** -10, 3 * 2 ** -10, -0.0,
                  -2 ** -11, 416.0, 432.0]
    f8[1, :4] = [-448.0, 300.0, 2 ** -6, 17.0]
    return bf, f8


def test_quantise_matches_library_casts(orc):
    """The oracle's exhaustive nearest-code search equals torch's
    round-to-nearest-even casts (BF16, FP8-E4M3FN) applied to the binary32
    quotients, on cluster data, sparse rows and the hand-made edge rows."""
    from paper_2503_06737_amd import synth
    bf, f8 = _quant_edge_rows()
    data = [synth.gaussian_clusters(200, 300, 5, 0.1, 93), synth.sparse_uniform(100, 333, 0.2, 94),
            (synth.gaussian_clusters(50, 64, 3, 1.0, 95) * 1e-4).astype(np.float32)]
    for kind, edge in (("bf16", bf), ("fp8", f8)):
        for x in data + [edge]:
            q, sc = orc.quantise_rows(x, kind)
            qt, sct = synth.quantise_rows(x, kind)
            assert (sc.view(np.uint32) == sct.view(np.uint32)).all(), kind
            assert (q == qt).all(), (kind, np.argwhere(q != qt)[:4])


def test_quantise_hand_cases(orc):
    """Hand-worked codes of the edge rows (ties to even, sign of zero, clamp)."""
    bf, f8 = _quant_edge_rows()
    q, sc = orc.quantise_rows(bf, "bf16")
    assert sc.tolist() == [1.0, 1.0, 1.0]
    assert q[0, :8].tolist() == [0x3F80, 0x3F00, 0x3F02, 0xBF00, 0x3E80, 0x8000, 0x0000, 0x3F40]
    assert (q[2] == 0).all()
    q, sc = orc.quantise_rows(f8, "fp8")
    assert sc.tolist() == [1.0, 1.0, 1.0]
    # 448 = 0x7E; 1.0 = 0x38; 1.25 = 0x3A; 2^-10 -> 0; 3*2^-10 -> 2^-8 = code 2;
    # -0 -> 0x80; -2^-11 -> negative zero; 416 = 1.625*2^8 = 0x7D; 432 is halfway
    # between 416 (odd mantissa 5) and 448 (even mantissa 6): 448
    assert q[0, :10].tolist() == [0x7E, 0x38, 0x3A, 0xB8, 0x00, 0x02, 0x80, 0x80, 0x7D, 0x7E]
    # -448 = 0xFE; 2^-6 is the smallest normal, 0x08; 17 is halfway between
    # 16 = 0x58 (even) and 18 = 0x59: 16
    assert q[1, :4].tolist() == [0xFE, orc_fp8_code(300.0), 0x08, 0x58]


def orc_fp8_code(v):
    """Code of the E4M3FN value nearest to v > 0 by a plain scan of the
    decoded values (ties cannot occur for the values used here)."""
    import oracle
    vals = [(abs(oracle.fp8_value(c) - v), c) for c in range(0x7F)]
    return min(vals)[1]


def test_quantise_decode_error_bound(orc):
    """Decoded values lie within half a code step of x: BF16 |err| <= 2^-9 |x|,
    FP8 normals |err| <= 2^-4 |x|, subnormals <= 2^-10 * scale."""
    from paper_2503_06737_amd import synth
    x = synth.gaussian_clusters(300, 256, 5, 0.2, 96)
    for kind in ("bf16", "fp8"):
        q, sc = orc.quantise_rows(x, kind)
        xd = orc.decode(q, sc)
        err = np.abs(xd - x.astype(np.float64))
        if kind == "bf16":
            bound = np.abs(x) * 2.0 ** -8 + 1e-38
        else:
            bound = np.maximum(np.abs(x) * 2.0 ** -4, 2.0 ** -10 * sc[:, None]) * (1 + 1e-6)
        assert (err <= bound).all(), kind


# ---------------------------------------------------------------------------
# independent per-table sketches (the protocol of Section 6)
# ---------------------------------------------------------------------------

def test_tables_worked_example(orc):
    """Hand-worked: two tables of K = 2 bins, scale sqrt(K) = sqrt(2), table t
    using shifts b[2t], b[2t+1] (tests/golden/tables_worked_example.json)."""
    g = json.load(open(os.path.join(GOLD, "tables_worked_example.json")))
    x = np.array([g["x"]])
    h = np.array(g["h"], np.uint32)
    s = np.array(g["s"], np.int8)
    b = np.array(g["b"], np.float32)
    out = orc.hash_points_tables(x, orc.E2LSH, g["K"], g["L"], kind="cs", w=g["w"], b=b, h=h, s=s)
    assert out["y"][0].tolist() == g["y"]
    assert out["codes"][0].tolist() == g["codes"]
    bits = orc.hash_points_tables(x, orc.SRP, g["K"], g["L"], kind="cs", h=h, s=s)
    assert bits["codes"][0].tolist() == g["srp_bits"]
    assert bits["keys"][:, 0].tolist() == [0b11, 0b00]


def test_tables_one_table_is_the_shared_sketch(orc):
    """Special case: with L = 1 the single table's sketch is the shared sketch
    of m = K components (same h, s, b, scale sqrt(K) = sqrt(m))."""
    gr = np.random.default_rng(101)
    x = gr.standard_normal((40, 37))
    K = 8
    h, s = gr.integers(0, K, 37).astype(np.uint32), gr.choice([-1, 1], 37).astype(np.int8)
    b = (gr.random(K) * 4).astype(np.float32)
    for fam in (orc.E2LSH, orc.SRP):
        a = orc.hash_points_tables(x, fam, K, 1, kind="cs", w=4.0, b=b, h=h[None], s=s[None])
        c = orc.hash_points(x, fam, K, 1, kind="cs", w=4.0, b=b, h=h, s=s)
        assert (a["codes"] == c["codes"]).all() and (a["keys"] == c["keys"]).all()


def test_tables_are_independent_and_ordered(orc):
    """Invariant: table t depends on its own state and shifts only.  Changing
    table u's hashes leaves every other table's sketch and key unchanged, and
    permuting the tables (state and shift blocks together) permutes the keys;
    a wrong table offset or shift block fails this."""
    gr = np.random.default_rng(102)
    n, d, K, L = 30, 50, 4, 5
    x = gr.standard_normal((n, d))
    h = gr.integers(0, K, (L, d)).astype(np.uint32)
    s = gr.choice([-1, 1], (L, d)).astype(np.int8)
    b = (gr.random(K * L) * 2).astype(np.float32)
    base = orc.hash_points_tables(x, orc.E2LSH, K, L, kind="cs", w=2.0, b=b, h=h, s=s)
    h2 = h.copy()
    h2[3] = gr.integers(0, K, d)
    alt = orc.hash_points_tables(x, orc.E2LSH, K, L, kind="cs", w=2.0, b=b, h=h2, s=s)
    keep = [t for t in range(L) if t != 3]
    assert (alt["keys"][keep] == base["keys"][keep]).all()
    assert (alt["y"][:, 12:16] != base["y"][:, 12:16]).any()
    perm = np.array([2, 0, 4, 1, 3])
    bp = b.reshape(L, K)[perm].reshape(-1)
    pr = orc.hash_points_tables(x, orc.E2LSH, K, L, kind="cs", w=2.0, b=bp, h=h[perm], s=s[perm])
    # table t of the permuted set is table perm[t] of the original, but its
    # key is seeded with its own index t: compare the codes, not the keys
    for t in range(L):
        assert (pr["codes"][:, t * K:(t + 1) * K] ==
                base["codes"][:, perm[t] * K:(perm[t] + 1) * K]).all()


def test_tables_hcs_is_cs_under_each_tables_composite_hash(orc):
    """Per-table HCS equals per-table CS when each table's composite bin and
    sign (first mode fastest) are given as its CS state."""
    gr = np.random.default_rng(103)
    dk, mk, L = (4, 3, 5), (2, 2, 2), 3
    d = 4 * 3 * 5
    K = 8
    x = gr.standard_normal((25, d))
    hk = [[gr.integers(0, m, dd).astype(np.uint32) for dd, m in zip(dk, mk)] for _ in range(L)]
    sk = [[gr.choice([-1, 1], dd).astype(np.int8) for dd in dk] for _ in range(L)]
    hc = np.zeros((L, d), np.uint32)
    sc = np.zeros((L, d), np.int8)
    for t in range(L):
        for j in range(d):
            i1, i2, i3 = j % 4, (j // 4) % 3, j // 12
            hc[t, j] = hk[t][0][i1] + 2 * (hk[t][1][i2] + 2 * hk[t][2][i3])
            sc[t, j] = sk[t][0][i1] * sk[t][1][i2] * sk[t][2][i3]
    b = (gr.random(K * L) * 4).astype(np.float32)
    a = orc.hash_points_tables(x, orc.E2LSH, K, L, kind="hcs", w=4.0, b=b, dk=dk, mk=mk, hk=hk, sk=sk)
    c = orc.hash_points_tables(x, orc.E2LSH, K, L, kind="cs", w=4.0, b=b, h=hc, s=sc)
    np.testing.assert_allclose(a["y"], c["y"], rtol=0, atol=1e-12)
    assert (a["keys"] == c["keys"]).all()
