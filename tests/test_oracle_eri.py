"""Pins for the oracle's contracted ERIs (Eq. 2, Section 2.2).

Each pin is independent of the oracle's McMurchie-Davidson code:
  * the closed form of [ss|ss] with scipy's erf;
  * every primitive p, d (and one f) integral as centre derivatives of that
    closed form, x_A^n exp(-a x_A^2) = O_n(d/dA_x) exp(-a x_A^2) with
    O_0 = 1, O_{n+1} = (d O_n + n O_{n-1}) / (2a), differentiated by mpmath
    at 30 digits;
  * Eq. 2's contraction as a sum of primitive blocks;
  * the eight-fold permutational symmetry, translation and rotation
    invariance, the Schwarz inequality, a positive semidefinite supermatrix
    and the far-field limit S_ab S_cd / R.
A dropped term, a wrong sign, a swapped index or operand in the oracle fails
at least one of them.
"""
import itertools
import math

import mpmath
import numpy as np
import pytest
from scipy.special import erf

import oracle
from paper_2412_13203_amd import inputs



def prim_basis(centres, exps, ls):
    """Four (or fewer) uncontracted shells with coefficient 1: raw primitives."""
    n = len(ls)
    return {
        "xyz": np.array(centres, dtype=np.float64),
        "shell_atom": np.arange(n, dtype=np.int32),
        "shell_l": np.array(ls, dtype=np.int32),
        "shell_nprim": np.ones(n, dtype=np.int32),
        "shell_prim_off": np.arange(n, dtype=np.int32),
        "exps": np.array(exps, dtype=np.float64),
        "coefs": np.ones(n, dtype=np.float64),
        "nbf": int(sum(inputs.ncart(l) for l in ls)),
    }


def ssss_closed(A, B, C, D, a, b, c, d):
    A, B, C, D = map(np.asarray, (A, B, C, D))
    p, q = a + b, c + d
    P = (a * A + b * B) / p
    Q = (c * C + d * D) / q
    rho = p * q / (p + q)
    T = rho * np.sum((P - Q) ** 2)
    F0 = 1.0 if T == 0 else 0.5 * math.sqrt(math.pi / T) * erf(math.sqrt(T))
    return (2 * math.pi ** 2.5 / (p * q * math.sqrt(p + q)) * math.exp(-a * b / p * np.sum((A - B) ** 2))
            * math.exp(-c * d / q * np.sum((C - D) ** 2)) * F0)


def _ssss_mp(x, ex):
    # x: 12 coordinates (A, B, C, D), ex: 4 exponents; mpmath closed form
    a, b, c, d = ex
    A, B, C, D = x[0:3], x[3:6], x[6:9], x[9:12]
    p, q = a + b, c + d
    P = [(a * A[i] + b * B[i]) / p for i in range(3)]
    Q = [(c * C[i] + d * D[i]) / q for i in range(3)]
    rho = p * q / (p + q)
    T = rho * sum((P[i] - Q[i]) ** 2 for i in range(3))
    AB2 = sum((A[i] - B[i]) ** 2 for i in range(3))
    CD2 = sum((C[i] - D[i]) ** 2 for i in range(3))
    F0 = mpmath.sqrt(mpmath.pi / T) / 2 * mpmath.erf(mpmath.sqrt(T))
    return (2 * mpmath.pi ** mpmath.mpf(2.5) / (p * q * mpmath.sqrt(p + q)) * mpmath.exp(-a * b / p * AB2)
            * mpmath.exp(-c * d / q * CD2) * F0)


def _op_poly(n, alpha):
    """Coefficients of O_n as a polynomial in d/dA (index = derivative order)."""
    polys = [[mpmath.mpf(1)]]
    if n >= 1:
        polys.append([mpmath.mpf(0), 1 / (2 * alpha)])
    for k in range(1, n):
        dOk = [mpmath.mpf(0)] + polys[k]
        prev = polys[k - 1] + [mpmath.mpf(0)] * (len(dOk) - len(polys[k - 1]))
        polys.append([(dOk[i] + k * prev[i]) / (2 * alpha) for i in range(len(dOk))])
    return polys[n]


def prim_eri_by_derivatives(centres, exps, cart):
    """[ab|cd] for Cartesian exponent triples cart[k] = (i, j, k) on centre k."""
    with mpmath.workdps(30):
        return _prim_eri_by_derivatives(centres, exps, cart)


def _prim_eri_by_derivatives(centres, exps, cart):
    x0 = [mpmath.mpf(v) for c in centres for v in c]
    ex = [mpmath.mpf(v) for v in exps]
    polys = []
    for k in range(4):
        for ax in range(3):
            polys.append(_op_poly(cart[k][ax], ex[k]))
    total = mpmath.mpf(0)
    for orders in itertools.product(*[range(len(p)) for p in polys]):
        coef = mpmath.mpf(1)
        for p, o in zip(polys, orders):
            coef *= p[o]
        if coef == 0:
            continue
        f = lambda *x: _ssss_mp(x, ex)  # noqa: E731
        total += coef * mpmath.diff(f, x0, orders)
    return float(total)


RNG = np.random.default_rng(20241213)


def _rand_geom(rng, n=4, box=2.0):
    return rng.uniform(-box / 2, box / 2, size=(n, 3))


def test_ssss_closed_form():
    rng = np.random.default_rng(1)
    for _ in range(20):
        cen = _rand_geom(rng)
        ex = np.exp(rng.uniform(np.log(0.1), np.log(50), size=4))
        b = prim_basis(cen, ex, [0, 0, 0, 0])
        v = oracle.eri_block(b, 0, 1, 2, 3)[0, 0, 0, 0]
        ref = ssss_closed(*cen, *ex)
        assert abs(v - ref) <= 1e-14 * abs(ref)


def test_ssss_coincident_centres():
    # T = 0: F_0 = 1
    cen = np.zeros((4, 3))
    ex = [0.7, 1.3, 0.4, 2.2]
    b = prim_basis(cen, ex, [0, 0, 0, 0])
    v = oracle.eri_block(b, 0, 1, 2, 3)[0, 0, 0, 0]
    assert abs(v - ssss_closed(*cen, *ex)) <= 1e-14 * v


CLASSES = [(1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1), (1, 1, 0, 0), (1, 0, 1, 0), (0, 1, 0, 1),
           (2, 0, 0, 0), (0, 2, 0, 0), (0, 0, 0, 2), (2, 1, 0, 0), (1, 1, 1, 0), (2, 0, 1, 0), (1, 1, 1, 1),
           (2, 2, 0, 0), (2, 0, 2, 0), (2, 1, 1, 0), (3, 0, 0, 0), (2, 2, 1, 1)]


@pytest.mark.parametrize("ls", CLASSES, ids=lambda t: "".join("spdf"[x] for x in t))
def test_primitive_by_centre_derivatives(ls):
    rng = np.random.default_rng(hash(ls) % 2 ** 32)
    cen = _rand_geom(rng, box=1.6)
    ex = np.exp(rng.uniform(np.log(0.3), np.log(3.0), size=4))
    b = prim_basis(cen, ex, list(ls))
    blk = oracle.eri_block(b, 0, 1, 2, 3)
    comps = [inputs.cart_components(l) for l in ls]
    idx = list(itertools.product(*[range(len(c)) for c in comps]))
    rng.shuffle(idx)
    nsample = 4 if sum(ls) >= 5 else 8
    for ii in idx[:nsample]:
        cart = [comps[k][ii[k]] for k in range(4)]
        ref = prim_eri_by_derivatives(cen, ex, cart)
        assert abs(blk[ii] - ref) <= 1e-12 * max(1.0, abs(ref)), (ls, cart, blk[ii], ref)


def test_contraction_is_sum_of_primitives():
    """Eq. 2: (ab|cd) = sum c_ak c_bl c_cm c_dn [a_k b_l|c_m d_n]."""
    rng = np.random.default_rng(7)
    basis = inputs.random_shells(rng, 4, [0], nprim_range=(2, 3))
    # take one shell per atom with l = (1, 2, 0, 1) by rebuilding four shells
    ls = [1, 2, 0, 1]
    cen = basis["xyz"]
    exps, coefs = [], []
    for k in range(4):
        n = 2 + (k % 2)
        exps.append(np.exp(rng.uniform(np.log(0.2), np.log(4), size=n)))
        coefs.append(rng.uniform(0.1, 1, size=n))
    contracted = {
        "xyz": cen, "shell_atom": np.arange(4, dtype=np.int32), "shell_l": np.array(ls, dtype=np.int32),
        "shell_nprim": np.array([len(e) for e in exps], dtype=np.int32),
        "shell_prim_off": np.array(np.cumsum([0] + [len(e) for e in exps[:-1]]), dtype=np.int32),
        "exps": np.concatenate(exps), "coefs": np.concatenate(coefs), "nbf": 0,
    }
    blk = oracle.eri_block(contracted, 0, 1, 2, 3)
    acc = np.zeros_like(blk)
    for ks in itertools.product(*[range(len(e)) for e in exps]):
        pb = prim_basis(cen, [exps[k][ks[k]] for k in range(4)], ls)
        c = np.prod([coefs[k][ks[k]] for k in range(4)])
        acc += c * oracle.eri_block(pb, 0, 1, 2, 3)
    assert np.max(np.abs(blk - acc)) <= 1e-14 * np.max(np.abs(blk))


def _random_basis(seed, ls=(0, 1, 2), natom=3):
    rng = np.random.default_rng(seed)
    return inputs.random_shells(rng, natom, list(ls), box=2.5, nprim_range=(1, 3), exp_range=(0.2, 6.0))


def test_eightfold_symmetry():
    b = _random_basis(11)
    ns = len(b["shell_l"])
    rng = np.random.default_rng(3)
    for _ in range(12):
        A, B, C, D = rng.integers(0, ns, size=4)
        ref = oracle.eri_block(b, A, B, C, D)
        assert np.allclose(oracle.eri_block(b, B, A, C, D), ref.transpose(1, 0, 2, 3), rtol=0, atol=1e-14)
        assert np.allclose(oracle.eri_block(b, A, B, D, C), ref.transpose(0, 1, 3, 2), rtol=0, atol=1e-14)
        assert np.allclose(oracle.eri_block(b, C, D, A, B), ref.transpose(2, 3, 0, 1), rtol=0, atol=1e-14)
        assert np.allclose(oracle.eri_block(b, D, C, B, A), ref.transpose(3, 2, 1, 0), rtol=0, atol=1e-14)


def test_translation_invariance():
    b = _random_basis(12)
    b2 = dict(b)
    b2["xyz"] = b["xyz"] + np.array([3.7, -1.2, 0.45])
    ns = len(b["shell_l"])
    for A, B, C, D in [(0, 1, 2, 3), (2, 5, 8, 4), (8, 8, 5, 5), (1, 2, 5, 8)]:
        A, B, C, D = [x % ns for x in (A, B, C, D)]
        assert np.allclose(oracle.eri_block(b, A, B, C, D), oracle.eri_block(b2, A, B, C, D), rtol=0, atol=1e-13)


def _cart_rotation(l, R):
    """Matrix T with phi'_m = sum_n T[m, n] phi_n for the l-shell under r -> R r."""
    comps = inputs.cart_components(l)
    index = {c: i for i, c in enumerate(comps)}
    T = np.zeros((len(comps), len(comps)))
    for m, c in enumerate(comps):
        # phi'_m = prod over the l factors (R u)_{axis}
        axes = [0] * c[0] + [1] * c[1] + [2] * c[2]
        for choice in itertools.product(range(3), repeat=l):
            coef = 1.0
            for ax, ch in zip(axes, choice):
                coef *= R[ax, ch]
            e = [0, 0, 0]
            for ch in choice:
                e[ch] += 1
            T[m, index[tuple(e)]] += coef
    return T


def test_rotation_invariance():
    b = _random_basis(13, ls=(1, 2, 0))
    rng = np.random.default_rng(5)
    Qm, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Qm) < 0:
        Qm[:, 0] *= -1
    b2 = dict(b)
    b2["xyz"] = b["xyz"] @ Qm.T
    ns = len(b["shell_l"])
    for quartet in [(0, 1, 3, 4), (1, 1, 4, 7), (4, 1, 7, 3), (6, 7, 1, 3), (2, 4, 5, 7)]:
        A, B, C, D = [x % ns for x in quartet]
        ref = oracle.eri_block(b, A, B, C, D)
        rot = oracle.eri_block(b2, A, B, C, D)
        Ts = [_cart_rotation(int(b["shell_l"][s]), Qm) for s in (A, B, C, D)]
        pred = np.einsum("ai,bj,ck,dl,ijkl->abcd", *Ts, ref)
        assert np.allclose(rot, pred, rtol=0, atol=1e-12), quartet


def test_schwarz_inequality():
    b = _random_basis(14)
    Q = oracle.schwarz(b)
    ns = len(b["shell_l"])
    rng = np.random.default_rng(9)
    for _ in range(15):
        A, B, C, D = rng.integers(0, ns, size=4)
        blk = oracle.eri_block(b, A, B, C, D)
        assert np.max(np.abs(blk)) <= Q[A, B] * Q[C, D] * (1 + 1e-12)
        dab = oracle.eri_block(b, A, B, A, B)
        dcd = oracle.eri_block(b, C, D, C, D)
        na, nb = blk.shape[:2]
        nc, nd = blk.shape[2:]
        diag_ab = np.array([[dab[i, j, i, j] for j in range(nb)] for i in range(na)])
        diag_cd = np.array([[dcd[i, j, i, j] for j in range(nd)] for i in range(nc)])
        bound = np.sqrt(np.einsum("ab,cd->abcd", diag_ab, diag_cd))
        assert np.all(np.abs(blk) <= bound * (1 + 1e-12) + 1e-300)


def test_supermatrix_psd_config1():
    cfg = inputs.make_config(1)
    T = oracle.eri_tensor(cfg["basis"])
    N = T.shape[0]
    M = T.reshape(N * N, N * N)
    assert np.allclose(M, M.T, rtol=0, atol=1e-13)
    w = np.linalg.eigvalsh(0.5 * (M + M.T))
    assert w.min() >= -1e-12 * w.max()


def test_far_field():
    # s shells on two atoms 400 bohr apart: (ab|cd) -> S_ab S_cd / R
    R = 400.0
    cen = [[0, 0, 0], [0.3, 0, 0], [R, 0, 0], [R, 0.2, 0]]
    b = prim_basis(cen, [1.1, 0.8, 0.9, 1.7], [0, 0, 0, 0])
    v = oracle.eri_block(b, 0, 1, 2, 3)[0, 0, 0, 0]
    Sab = oracle.overlap_block(b, 0, 1)[0, 0]
    Scd = oracle.overlap_block(b, 2, 3)[0, 0]
    Rpq = np.linalg.norm((1.1 * np.array(cen[0]) + 0.8 * np.array(cen[1])) / 1.9
                         - (0.9 * np.array(cen[2]) + 1.7 * np.array(cen[3])) / 2.6)
    assert abs(v - Sab * Scd / Rpq) <= 1e-12 * v


def test_normalization_of_input_recipe():
    """x^l component has unit self-overlap; d_xy has 1/3 (shared factor)."""
    cfg = inputs.make_config(2, natom=2)
    b = cfg["basis"]
    for s in range(len(b["shell_l"])):
        S = oracle.overlap_block(b, s, s)
        assert abs(S[0, 0] - 1.0) < 1e-13
        if b["shell_l"][s] == 2:
            assert abs(S[1, 1] - 1.0 / 3.0) < 1e-13


def test_overlap_closed_form():
    # two s primitives: (pi/p)^{3/2} exp(-ab/p R^2)
    cen = [[0, 0, 0], [0.4, -0.3, 1.1]]
    b = prim_basis(cen, [0.9, 2.3], [0, 0])
    S = oracle.overlap_block(b, 0, 1)[0, 0]
    p = 3.2
    R2 = 0.16 + 0.09 + 1.21
    assert abs(S - (math.pi / p) ** 1.5 * math.exp(-0.9 * 2.3 / p * R2)) < 1e-15


def test_schwarz_value_is_sqrt_of_largest_diagonal():
    """Pins orc_schwarz's value, not only its bound: Q_AB = sqrt(max over the
    components a in A, b in B of the diagonal integral (ab|ab)), for every
    shell pair of a small s, p, d basis (the contracted blocks come from
    eri_block, itself pinned above).  A sum in place of the max, an
    off-diagonal element or a missing square root fails here; the basis is
    rescaled so that some diagonal integrals exceed 1, where a missing
    square root would otherwise hide behind values below 1."""
    b = _random_basis(21, ls=(0, 1, 2), natom=3)
    b = dict(b)
    b["coefs"] = np.asarray(b["coefs"]) * 3.0
    Q = oracle.schwarz(b)
    ns = len(b["shell_l"])
    assert np.array_equal(Q, Q.T)
    above_one = 0
    for A in range(ns):
        for B in range(A + 1):
            blk = oracle.eri_block(b, A, B, A, B)
            na, nb = blk.shape[:2]
            diag = np.array([blk[i, j, i, j] for i in range(na) for j in range(nb)])
            assert np.all(diag > 0)
            above_one += int(diag.max() > 1.0)
            ref = math.sqrt(float(diag.max()))
            assert abs(Q[A, B] - ref) <= 1e-15 * ref, (A, B, Q[A, B], ref)
    assert above_one > 0


def test_schwarz_closed_form_primitives():
    """Pins orc_schwarz against the closed form, independently of the oracle's
    integrals: for single primitives with coefficient c, Q_AB^2 is
    c_a^2 c_b^2 [ab|ab]; for two s shells that is the [ss|ss] closed form,
    and for a p shell on A and an s shell on B it is the largest of the three
    [p_i s|p_i s], each a centre derivative of the closed form (mpmath).
    The coefficients make the values exceed 1."""
    rng = np.random.default_rng(33)
    for _ in range(3):
        cen = _rand_geom(rng, n=2, box=1.5)
        ex = np.exp(rng.uniform(np.log(0.3), np.log(4.0), size=2))
        ca, cb = 2.5, 1.7
        # s s
        bs = prim_basis(cen, ex, (0, 0))
        bs["coefs"] = np.array([ca, cb])
        Q = oracle.schwarz(bs)
        ref = ca * cb * math.sqrt(ssss_closed(cen[0], cen[1], cen[0], cen[1], ex[0], ex[1], ex[0], ex[1]))
        assert ref > 1.0
        assert abs(Q[0, 1] - ref) <= 1e-13 * ref
        # p s: max over the three components of [p_i s | p_i s]
        bp = prim_basis(cen, ex, (1, 0))
        bp["coefs"] = np.array([ca, cb])
        Qp = oracle.schwarz(bp)
        four = [cen[0], cen[1], cen[0], cen[1]]
        exs = [ex[0], ex[1], ex[0], ex[1]]
        vals = []
        for i in range(3):
            e = [0, 0, 0]
            e[i] = 1
            vals.append(prim_eri_by_derivatives(four, exs, [tuple(e), (0, 0, 0), tuple(e), (0, 0, 0)]))
        refp = ca * cb * math.sqrt(max(vals))
        assert abs(Qp[0, 1] - refp) <= 1e-11 * refp, (Qp[0, 1], refp)
