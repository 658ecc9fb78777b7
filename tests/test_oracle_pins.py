"""Pins for the CPU oracle: it is checked against what the paper and the
mathematics fix, never against itself.

* rounding helpers vs numpy/torch conversions and the paper's Table 1;
* exact summation and residuals vs rational arithmetic;
* Algorithm 1 closed forms: diagonal and permutation matrices, full pattern;
* fixed-pattern columns vs the least-squares definition (numpy lstsq and
  exact rational normal equations);
* candidate scores vs brute-force univariate minimisation, selection rule,
  monotonicity and the Frobenius/infinity-norm bounds of Section 3.1;
* GMRES vs the exact Krylov least-squares minimiser, the exact-preconditioner
  case of Table 5, and the limiting accuracy of Theorems 1-2.
"""
import math
import random
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W

GOLDEN = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden")


def _csr(dense):
    S = sp.csr_matrix(dense)
    S.sort_indices()
    S.eliminate_zeros()
    return W.CSR(S.shape[0], S.indptr.astype(np.int32), S.indices.astype(np.int32),
                 S.data.astype(np.float64))


def _dense(A):
    return A.to_scipy().toarray()


def _random_dd(n, rng, density=0.3, dom=1.5):
    """random nonsymmetric, nonzero diagonal, row diagonally dominant"""
    M = rng.standard_normal((n, n)) * (rng.random((n, n)) < density)
    np.fill_diagonal(M, 0.0)
    np.fill_diagonal(M, dom * np.abs(M).sum(1) + 1.0)
    M *= np.where(rng.random(n) < 0.5, -1.0, 1.0)[:, None]   # random row signs
    return M


# ---------------------------------------------------------------------------
# precision helpers
# ---------------------------------------------------------------------------

def _special_f32(rng, count):
    vals = list(rng.standard_normal(count // 2) * 10.0 ** rng.integers(-9, 6, count // 2))
    vals += list(np.ldexp(rng.integers(-2**23, 2**23, count // 2).astype(np.float64), -30))
    vals += [0.0, -0.0, 65504.0, 65519.99, 65520.0, -65520.0, 6.1e-5, 5.96e-8, 2.98e-8, 1e-9,
             3.0e38, 1.2e-38, 1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11]
    return np.array(vals, dtype=np.float32).astype(np.float64)


def test_round_fp16_matches_numpy_conversion():
    xs = _special_f32(np.random.default_rng(1), 20000)
    ours = np.array([O.round_to(x, "fp16") for x in xs])
    ref = xs.astype(np.float32).astype(np.float16).astype(np.float64)
    assert np.array_equal(ours, ref, equal_nan=True)


def test_round_bf16_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    xs = _special_f32(np.random.default_rng(2), 20000)
    xs = xs[np.abs(xs) < 3.0e38]
    ours = np.array([O.round_to(x, "bf16") for x in xs])
    ref = torch.tensor(xs, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)


def test_unit_roundoff_matches_table1():
    """Max relative rounding error over normal values equals the printed u."""
    table = {}
    for line in open(f"{GOLDEN}/table1_unit_roundoff.txt"):
        if line.strip() and not line.startswith("#"):
            name, _bits, e = line.split()
            table[name] = 2.0 ** int(e)
    rng = np.random.default_rng(3)
    xs = np.exp(rng.uniform(-5, 5, 50000))
    for name, uf in (("half", "fp16"), ("single", "fp32")):
        rel = max(abs(O.round_to(x, uf) - x) / abs(x) for x in xs)
        u = table[name]
        assert rel <= u * (1 + 1e-12)
        assert rel > 0.9 * u, (name, rel, u)


# ---------------------------------------------------------------------------
# exact summation and residual
# ---------------------------------------------------------------------------

def test_exact_sum_vs_fsum_and_fractions():
    rng = random.Random(4)
    for _ in range(300):
        k = rng.randint(1, 40)
        xs = [rng.choice([1, -1]) * rng.random() * 2.0 ** rng.randint(-60, 60) for _ in range(k)]
        xs += [-x for x in xs[: rng.randint(0, k)]]        # cancellation
        xs.append(rng.random() * 2.0 ** -80)
        rng.shuffle(xs)
        exact = float(sum(Fraction(x) for x in xs))         # Fraction -> float rounds correctly
        assert O.exact_sum(xs) == exact == math.fsum(xs)
    for _ in range(300):                                    # subnormals, extreme exponents, ties
        k = rng.randint(1, 12)
        xs = [rng.choice([1, -1]) * rng.randint(1, 2 ** 53 - 1) * 2.0 ** rng.randint(-1126, 960)
              for _ in range(k)]
        xs += [rng.choice([1, -1]) * 2.0 ** -1074 * rng.randint(1, 9)]
        if rng.random() < 0.5:                              # a halfway case: 1 + 2^-53 (+ tiny)
            xs += [1.0, 2.0 ** -53] + ([2.0 ** -1000] if rng.random() < 0.5 else [])
        rng.shuffle(xs)
        exact = float(sum(Fraction(x) for x in xs))
        assert O.exact_sum(xs) == exact, xs


def test_residual_is_exactly_rounded():
    rng = np.random.default_rng(5)
    for n in (7, 23):
        A = _csr(_random_dd(n, rng))
        x = rng.standard_normal(n)
        b = rng.standard_normal(n)
        r = O.residual(A, b, x)
        D = _dense(A)
        for i in range(n):
            exact = Fraction(b[i]) - sum(Fraction(D[i, j]) * Fraction(x[j]) for j in range(n) if D[i, j] != 0)
            assert r[i] == float(exact)


@pytest.mark.parametrize("make", [lambda: W.convdiff_small(32), lambda: W.convdiff_adaptive(24),
                                  lambda: W.aniso_fixed(8), lambda: W.random_system(300)])
def test_exact_rhs_has_zero_residual(make):
    w = make()
    assert np.all(O.residual(w.A, w.b, w.x_true) == 0.0)


# ---------------------------------------------------------------------------
# Algorithm 1: closed forms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("uf", ["fp64", "fp32", "fp16", "bf16"])
def test_diagonal_matrix_gives_exact_inverse(uf):
    """B = A^T D is diagonal with B_kk = d_k a_kk, within one FP64 rounding of
    sign(a_kk); rounded to a u_f coarser than FP64 it is +-1 exactly, so m-bar =
    +-1, the residual is 0 and P = diag(d_k sign(a_kk)) = diag(fl(1/a_kk)).
    Extra pattern entries get exactly zero coefficients."""
    rng = np.random.default_rng(6)
    n = 40
    diag = rng.uniform(0.1, 50.0, n) * np.where(rng.random(n) < 0.5, -1, 1)
    A = _csr(np.diag(diag))
    for pattern in (None, W.pattern_of(_csr(np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)))):
        R = O.spai(A, pattern, eps=0.1, alpha=5, beta=8, maxfill=8, uf=uf)
        assert np.all(R.steps == 0) and np.all(R.flags == 0)
        pp, pc, pv = R.P_csr(n)
        Pd = sp.csr_matrix((pv * R.d[pc], pc, pp), shape=(n, n)).toarray()
        assert np.count_nonzero(Pd - np.diag(np.diag(Pd))) == 0
        if uf == "fp64":
            assert np.all(R.res <= 2.0 ** -52)
            assert np.all(np.abs(np.diag(Pd) * diag - 1.0) <= 4 * 2.0 ** -53)
        else:
            assert np.all(R.res == 0.0)
            assert np.array_equal(np.diag(Pd), 1.0 / diag)


@pytest.mark.parametrize("uf", ["fp64", "fp32", "fp16"])
def test_permutation_matrix_closed_form_trace(uf):
    """Identity start on a permutation matrix: fixed points stop at step 0 with
    m-bar = 1; every other column finds its single candidate j* = pi^{-1}(k) with
    rho = 0 = rho-bar, stops after one augmentation with J_k = (k, j*), m-bar =
    (0, 1), residual 0, and P A = I exactly.  This pins the residual on the full
    column (k outside the shadow contributes 1) and the full-column score."""
    rng = np.random.default_rng(7)
    n = 60
    perm = np.arange(n)
    perm[5:] = 5 + rng.permutation(n - 5)       # 0..4 (and maybe more) are fixed points
    Pm = np.zeros((n, n))
    Pm[np.arange(n), perm] = 1.0                # A(k, pi(k)) = 1
    A = _csr(Pm)
    R = O.spai(A, None, eps=0.2, alpha=-(-n // 8), beta=8, maxfill=10, uf=uf)
    inv = np.argsort(perm)                       # pi^{-1}
    for k in range(n):
        if perm[k] == k:
            assert R.steps[k] == 0 and R.length[k] == 1 and R.m[k, 0] == 1.0
        else:
            assert R.steps[k] == 1 and R.length[k] == 2
            assert list(R.J[k, :2]) == [k, inv[k]]
            assert R.m[k, 0] == 0.0 and R.m[k, 1] == 1.0
        assert R.res[k] == 0.0
    pp, pc, pv = R.P_csr(n)
    PA = sp.csr_matrix((pv * R.d[pc], pc, pp), shape=(n, n)) @ A.to_scipy()
    assert np.array_equal(PA.toarray(), np.eye(n))


@pytest.mark.parametrize("uf,tol", [("fp64", 1e-12), ("fp32", 2e-4)])
def test_full_pattern_reproduces_dense_inverse(uf, tol):
    """With J = all indices each column solves B m_k = e_k exactly (Section 3.1
    notes the full-pattern limit), so P = M^T D = A^{-1}."""
    rng = np.random.default_rng(8)
    n = 30
    Ad = _random_dd(n, rng, density=0.4)
    A = _csr(Ad)
    full = W.Pattern(n, np.arange(0, n * n + 1, n, dtype=np.int32), np.tile(np.arange(n, dtype=np.int32), n))
    R = O.spai(A, full, eps=1e-30, alpha=0, beta=8, maxfill=n, uf=uf)
    pp, pc, pv = R.P_csr(n)
    P = sp.csr_matrix((pv * R.d[pc], pc, pp), shape=(n, n)).toarray()
    Ainv = np.linalg.inv(Ad)
    err = np.abs(P - Ainv).max() / np.abs(Ainv).max()
    kappa = np.linalg.cond(Ad, 1)
    assert err <= tol * max(1.0, kappa / 10.0), (err, kappa)


# ---------------------------------------------------------------------------
# fixed-pattern columns vs the least-squares definition
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("uf", ["fp64", "fp32", "fp16"])
def test_power_of_two_row_scaling_leaves_M_unchanged(uf):
    """Section 4's scaling D = diag(1 / max_j |a_ij|) absorbs any row scaling of A
    by powers of two exactly: B = (S A)^T D' = A^T D with D' = D S^-1, so Algorithm 1
    sees the same B and returns the same M bit for bit (adaptive pattern included),
    while d scales by 2^-k_i.  A scaling taken from the columns, or applied on the
    other side of A, breaks this; scaling the columns instead does change M."""
    rng = np.random.default_rng(21)
    n = 48
    Ad = _random_dd(n, rng, density=0.12)
    k = rng.integers(-8, 9, n)
    R = O.spai(_csr(Ad), None, 0.2, 4, 3, 12, uf)
    R2 = O.spai(_csr(Ad * np.ldexp(1.0, k)[:, None]), None, 0.2, 4, 3, 12, uf)
    assert R.steps.max() >= 1                      # the adaptive path ran
    assert np.array_equal(R.length, R2.length) and np.array_equal(R.J, R2.J)
    assert np.array_equal(R.m, R2.m) and np.array_equal(R.res, R2.res)
    assert np.array_equal(R2.d, np.ldexp(R.d, -k))
    R3 = O.spai(_csr(Ad * np.ldexp(1.0, k)[None, :]), None, 0.2, 4, 3, 12, uf)
    assert not np.array_equal(R3.m, R.m)


def test_power_of_two_column_scaling_leaves_the_right_M_unchanged():
    """The right form scales the columns of A to unit maximum, so A S with
    S = diag(2^k_j) gives the same M (rows of P = D M scaled by 2^-k_i through d
    only) and the same A P."""
    rng = np.random.default_rng(22)
    n = 40
    Ad = _random_dd(n, rng, density=0.15)
    k = rng.integers(-8, 9, n)
    R, pp, pc, pv, d = O.spai_right(_csr(Ad), None, 0.25, 3, 4, 10, "fp32")
    R2, pp2, pc2, pv2, d2 = O.spai_right(_csr(Ad * np.ldexp(1.0, k)[None, :]), None, 0.25, 3, 4, 10, "fp32")
    assert np.array_equal(pp, pp2) and np.array_equal(pc, pc2) and np.array_equal(pv, pv2)
    assert np.array_equal(d2, np.ldexp(d, -k))
    P = np.diag(d) @ sp.csr_matrix((pv, pc, pp), shape=(n, n)).toarray()
    P2 = np.diag(d2) @ sp.csr_matrix((pv2, pc2, pp2), shape=(n, n)).toarray()
    assert np.array_equal(Ad @ P, (Ad * np.ldexp(1.0, k)[None, :]) @ P2)


@pytest.mark.parametrize("make", [lambda: W.convdiff_small(16), lambda: W.aniso_fixed(6)])
def test_fixed_pattern_fp64_matches_lstsq(make):
    w = make()
    A = w.A
    R = O.spai(A, w.pattern, eps=w.spai.eps, alpha=0, beta=8, maxfill=w.spai.maxfill, uf="fp64")
    worst = 0.0
    for k in range(A.n):
        L = R.length[k]
        J = R.J[k, :L]
        assert sorted(J) == sorted(w.pattern.idx[w.pattern.ptr[k]:w.pattern.ptr[k + 1]])
        mbar, res = O.ls_column(A, R.d, k, J)
        worst = max(worst, np.abs(R.m[k, :L] - mbar).max() / np.abs(mbar).max())
        assert abs(R.res[k] - res) <= 1e-12 * max(res, 1e-300) + 1e-15
    assert worst < 1e-12


def test_fixed_pattern_fp64_matches_exact_normal_equations():
    """Exact rational solution of (A-bar^T A-bar) m = A-bar^T e-bar on tiny inputs."""
    rng = np.random.default_rng(9)
    n = 9
    Ad = _random_dd(n, rng, density=0.35)
    A = _csr(Ad)
    pat = _csr((rng.random((n, n)) < 0.3) | np.eye(n, dtype=bool))
    pattern = W.Pattern(n, pat.rowptr, pat.col)
    R = O.spai(A, pattern, eps=1e-30, alpha=0, beta=8, maxfill=n, uf="fp64")
    d = O.scaling(A)
    for k in range(n):
        L = R.length[k]
        J = [int(j) for j in R.J[k, :L]]
        I = sorted({i for j in J for i in range(n) if Ad[j, i] != 0})
        Ab = [[Fraction(d[j] * Ad[j, i]) for j in J] for i in I]   # B(i, j) = d_j a_ji (FP64 product)
        e = [Fraction(int(i == k)) for i in I]
        p = len(J)
        G = [[sum(Ab[r][a] * Ab[r][b] for r in range(len(I))) for b in range(p)] for a in range(p)]
        h = [sum(Ab[r][a] * e[r] for r in range(len(I))) for a in range(p)]
        # Gauss-Jordan in exact arithmetic
        M = [row[:] + [h[a]] for a, row in enumerate(G)]
        for c in range(p):
            piv = next(r for r in range(c, p) if M[r][c] != 0)
            M[c], M[piv] = M[piv], M[c]
            M[c] = [v / M[c][c] for v in M[c]]
            for r in range(p):
                if r != c and M[r][c] != 0:
                    M[r] = [a - M[r][c] * b for a, b in zip(M[r], M[c])]
        exact = np.array([float(M[a][p]) for a in range(p)])
        kap = np.linalg.cond(np.array([[float(v) for v in row] for row in Ab]))
        assert np.abs(R.m[k, :L] - exact).max() <= 10 * kap * 2.0 ** -53 * np.abs(exact).max() * 10


# ---------------------------------------------------------------------------
# candidate scores, selection and invariants of the adaptive loop
# ---------------------------------------------------------------------------

def test_rho_is_the_univariate_minimum():
    """rho_j^2 = min_mu ||r - mu B e_j||^2 with r = e_k - B m_k on all n rows,
    and adding j alone to J leaves a residual no larger than rho_j."""
    w = W.convdiff_adaptive(12)
    A = w.A
    Bd = (_dense(A).T * O.scaling(A)[None, :])     # B = A^T D
    n = A.n
    rng = np.random.default_rng(10)
    for k in rng.choice(n, 25, replace=False):
        J = [int(k)]
        for _ in range(3):
            pr = O.spai_probe(A, int(k), J, "fp64")
            mfull = np.zeros(n)
            mfull[J] = pr.mbar
            r = np.eye(n)[:, k] - Bd @ mfull
            assert abs(np.linalg.norm(r) - pr.res) <= 1e-12
            for j, rho in zip(pr.cand, pr.rho):
                bj = Bd[:, j]
                mu = (r @ bj) / (bj @ bj)
                brute = np.linalg.norm(r - mu * bj)
                assert abs(brute - rho) <= 1e-10 * max(1.0, brute)
                pj = O.spai_probe(A, int(k), J + [int(j)], "fp64")
                assert pj.res <= rho + 1e-12
            assert abs(pr.rbar - pr.rho.mean()) <= 1e-12
            # every column index that meets the shadow's rows (or row k) is a candidate
            L = set(pr.I.tolist()) | {int(k)}
            cands = sorted({int(j) for j in range(n) if j not in J and any(Bd[l, j] != 0 for l in L)})
            assert list(pr.cand) == cands
            J = J + [int(pr.cand[np.argmin(pr.rho)])]


@pytest.mark.parametrize("uf", ["fp64", "fp32"])
def test_selection_rule_and_invariants(uf):
    """Replaying each column from its insertion-ordered J: every step adds the
    min(beta, |acceptable|, maxfill - |J|) acceptable candidates with the
    smallest (rho, j); residuals never increase (exact LS property, up to
    rounding); the stop happens at res <= eps, the fill cap or alpha."""
    w = W.convdiff_adaptive(16, u_f=uf)
    A, s = w.A, w.spai
    R = O.spai(A, None, s.eps, s.alpha, s.beta, s.maxfill, uf)
    u = 2.0 ** -53 if uf == "fp64" else 2.0 ** -24
    for k in range(0, A.n, 7):
        L = R.length[k]
        Jk = [int(j) for j in R.J[k, :L]]
        assert Jk[0] == k and len(set(Jk)) == L and L <= s.maxfill
        pos = 1
        hist = R.hist[k][~np.isnan(R.hist[k])]
        assert len(hist) == R.steps[k] + 1
        assert np.all(np.diff(hist) <= 1e3 * u)
        Iprev = None
        for step in range(R.steps[k]):
            pr = O.spai_probe(A, k, Jk[:pos], uf, Iprev=Iprev)
            assert pr.res == hist[step] and pr.res > s.eps
            # the shadow grows in insertion order: the previous rows keep their places
            if Iprev is not None:
                assert list(pr.I[:len(Iprev)]) == list(Iprev)
                assert list(pr.I[len(Iprev):]) == sorted(pr.I[len(Iprev):])
            Iprev = pr.I
            acc = sorted([(rho, j) for j, rho in zip(pr.cand, pr.rho) if rho <= pr.rbar])
            nsel = min(s.beta, len(acc), s.maxfill - pos)
            assert Jk[pos:pos + nsel] == [j for _, j in acc[:nsel]]
            pos += nsel
        assert pos == L
        if R.res[k] > s.eps:
            assert R.flags[k] & O.FLAG_EPS and (L >= s.maxfill or R.steps[k] >= s.alpha)


def test_frobenius_decoupling_and_bounds():
    """||I - B M||_F^2 = sum_k ||e_k - B m_k||^2 (eq. fronormmin), <= n eps^2 when
    every column meets eps, and ||I - P A||_inf <= 2 n eps (eq. AM1)."""
    w = W.convdiff_adaptive(20, u_f="fp64")
    A, s = w.A, w.spai
    R = O.spai(A, None, s.eps, s.alpha, s.beta, s.maxfill, "fp64")
    n = A.n
    assert np.all(R.res <= s.eps)
    pp, pc, pv = R.P_csr(n)
    M_T = sp.csr_matrix((pv, pc, pp), shape=(n, n))             # row k = m_k^T
    B = A.to_scipy().T @ sp.diags(R.d)
    E = (sp.identity(n) - B @ M_T.T).toarray()
    fro2 = (E ** 2).sum()
    assert abs(fro2 - (R.res ** 2).sum()) <= 1e-10 * fro2
    assert math.sqrt(fro2) <= math.sqrt(n) * s.eps
    PA = (M_T @ sp.diags(R.d) @ A.to_scipy()).toarray()
    assert np.abs(np.eye(n) - PA).sum(1).max() <= 2 * n * s.eps


def test_larger_eps_gives_sparser_preconditioner_and_more_iterations():
    """Section 4: a larger eps gives a sparser P and more GMRES iterations."""
    w = W.convdiff_adaptive(32)
    A, s, ir = w.A, w.spai, w.ir
    nnz, tot = [], []
    for eps in (0.5, 0.3, 0.2):
        R = O.spai(A, None, eps, s.alpha, s.beta, 40, "fp32")
        pp, pc, pv = R.P_csr(A.n)
        res = O.gmres_ir(A, pp, pc, pv, R.d, "fp32", w.b, ir.tau, ir.imax, ir.maxit, ir.tol_ir)
        nnz.append(pp[-1])
        tot.append(res.total)
        assert O.ferr(res.x, w.x_true) <= 1e-12
    assert nnz[0] < nnz[1] < nnz[2]
    assert tot[0] > tot[1] > tot[2]


def test_fp32_and_fp64_spai_give_similar_preconditioners():
    """Section 3.1 / Table 5: no benefit from u_f finer than the eps-dictated level."""
    w = W.convdiff_adaptive(32)
    A, s, ir = w.A, w.spai, w.ir
    out = {}
    for uf in ("fp32", "fp64"):
        R = O.spai(A, None, s.eps, s.alpha, s.beta, s.maxfill, uf)
        pp, pc, pv = R.P_csr(A.n)
        res = O.gmres_ir(A, pp, pc, pv, R.d, uf, w.b, ir.tau, ir.imax, ir.maxit, ir.tol_ir)
        out[uf] = (pp[-1], res.total)
    assert abs(out["fp32"][0] - out["fp64"][0]) <= 0.02 * out["fp64"][0]
    assert abs(out["fp32"][1] - out["fp64"][1]) <= 0.1 * out["fp64"][1]


# ---------------------------------------------------------------------------
# GMRES-IR
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ortho", ["mgs", "cgs2", "dcgs2"])
def test_gmres_step_is_the_krylov_least_squares_minimiser(ortho):
    """After k iterations (tau = 0) GMRES (MGS or CGS2 Arnoldi) returns
    d = argmin over K_k(PA, z) of ||z - PA d||_2 with z = P r0; checked against
    an orthonormal basis of the explicit Krylov matrix."""
    rng = np.random.default_rng(11)
    n = 8
    Ad = _random_dd(n, rng, density=0.6, dom=0.4)
    A = _csr(Ad)
    b = rng.standard_normal(n)
    for use_identity in (True, False):
        if use_identity:                                  # P = I: plain GMRES
            pp, pc, pv, d = np.arange(n + 1), np.arange(n), np.ones(n), np.ones(n)
        else:
            R = O.spai(A, None, 0.6, 0, 8, 8, "fp64")      # a diagonal P
            pp, pc, pv = R.P_csr(n)
            d = R.d
        P = sp.csr_matrix((pv * d[pc], pc, pp), shape=(n, n)).toarray()
        for k in range(1, 6):
            res = O.gmres_ir(A, pp, pc, pv, d, "fp64", b, 0.0, 1, k, 0.0, ortho)
            assert res.its == [k]
            x0 = P @ b
            r0 = b - Ad @ x0
            z = P @ r0
            PA = P @ Ad
            K = np.column_stack([np.linalg.matrix_power(PA, i) @ z for i in range(k)])
            Q, _ = np.linalg.qr(K)
            y, *_ = np.linalg.lstsq(PA @ Q, z, rcond=None)
            dexp = Q @ y
            assert np.abs((res.x - x0) - dexp).max() <= 1e-9 * np.abs(dexp).max()


def test_long_arnoldi_runs_stay_the_krylov_minimiser():
    """Over 10, 40 and 120 iterations (tau = 0) of one GMRES step with a
    non-diagonal SPAI P (n = 400), MGS, CGS2 and delayed CGS2 each return the
    minimiser of ||z - PA d||_2 over K_k(PA, z), z = P r0, against a basis built
    here by numpy (each new direction PA q_i projected out twice with matrix
    products, then normalised): a wrong index or lag in the delayed recurrences
    shows up after a few steps, which the short runs above cannot see."""
    w = W.convdiff_adaptive(20)
    s = w.spai
    R = O.spai(w.A, None, s.eps, s.alpha, s.beta, s.maxfill, "fp64")
    pp, pc, pv = R.P_csr(w.n)
    Ad = _dense(w.A)
    P = sp.csr_matrix((pv * R.d[pc], pc, pp), shape=(w.n, w.n)).toarray()
    PA = P @ Ad
    x0 = P @ w.b
    z = P @ (w.b - Ad @ x0)
    Q = np.zeros((w.n, 121))
    Q[:, 0] = z / np.linalg.norm(z)
    for i in range(120):
        v = PA @ Q[:, i]
        for _ in range(2):
            v -= Q[:, :i + 1] @ (Q[:, :i + 1].T @ v)
        Q[:, i + 1] = v / np.linalg.norm(v)
    for k in (10, 40, 120):
        y, *_ = np.linalg.lstsq(PA @ Q[:, :k], z, rcond=None)
        dexp = Q[:, :k] @ y
        for ortho in ("mgs", "cgs2", "dcgs2"):
            res = O.gmres_ir(w.A, pp, pc, pv, R.d, "fp64", w.b, 0.0, 1, k, 0.0, ortho)
            assert res.its == [k]
            err = np.abs((res.x - x0) - dexp).max() / np.abs(dexp).max()
            assert err <= 1e-9, (k, ortho, err)


def test_twice_projected_bases_stay_orthonormal():
    """Classical Gram-Schmidt applied twice keeps the Arnoldi basis orthonormal to
    working precision while the one-pass orthogonalisations lose it in
    proportion to the conditioning the iteration reaches (Giraud, Langou and
    Rozloznik, 2005; modified Gram-Schmidt's loss is what Section 3.2's analysis
    allows for).  On plain GMRES (P = I) over a convection-diffusion matrix,
    where MGS's basis has lost orthogonality completely by 70 iterations, the
    CGS2 and delayed-CGS2 bases stay within 1e-14 of orthonormal; the delayed
    scheme with its second projection removed (CGS1) fails this."""
    w = W.convdiff_adaptive(24)
    n = w.n
    pp, pc, pv, d = np.arange(n + 1), np.arange(n), np.ones(n), np.ones(n)
    loss = {}
    for ortho in ("mgs", "cgs2", "dcgs2"):
        for k in (40, 70, 90):
            V = O.gmres_ir(w.A, pp, pc, pv, d, "fp64", w.b, 0.0, 1, k, 0.0, ortho, basis=True).basis0
            assert V.shape == (n, k)
            loss[ortho, k] = float(np.abs(np.eye(k) - V.T @ V).max())
    assert loss["mgs", 40] <= 1e-9 and loss["mgs", 90] >= 0.1, loss
    for k in (40, 70, 90):
        assert loss["cgs2", k] <= 1e-14 and loss["dcgs2", k] <= 1e-14, loss


def test_exact_preconditioner_takes_one_iteration_per_step():
    """Table 5 prints 1(1) for the exact (full LU, u_f = u) preconditioner."""
    its_golden = int(open(f"{GOLDEN}/exact_preconditioner_its.txt").read().split("its_per_step")[1])
    w = W.convdiff_small(10)
    Ad = _dense(w.A)
    Ainv = np.linalg.inv(Ad)
    S = sp.csr_matrix(Ainv)
    S.sort_indices()
    res = O.gmres_ir(w.A, S.indptr, S.indices, S.data, np.ones(w.n), "fp64", w.b, 1e-8, 10, 50, W.TOL_IR)
    assert all(k == its_golden for k in res.its)
    assert len(res.its) <= 3
    assert O.ferr(res.x, w.x_true) <= 1e-15


def test_limiting_accuracy_convdiff_small():
    """Theorems 1-2: with u_r <= u^2 the forward error reaches ~u and the
    backward error ~q u (C1: FP32 SPAI on pattern(A), FP64 GMRES)."""
    w = W.convdiff_small(32)
    s, ir = w.spai, w.ir
    R = O.spai(w.A, w.pattern, s.eps, s.alpha, s.beta, s.maxfill, s.u_f)
    pp, pc, pv = R.P_csr(w.n)
    res = O.gmres_ir(w.A, pp, pc, pv, R.d, s.u_f, w.b, ir.tau, ir.imax, ir.maxit, ir.tol_ir)
    assert res.status & ~O.IR_STAGNATED == 0
    assert O.ferr(res.x, w.x_true) <= 1e-12
    assert O.nbe(w.A, w.b, res.x) <= 5 * 2.0 ** -53
    assert len(res.its) >= 2


def test_x0_in_fp32_is_sequential_fp32():
    """x0 = P b in u_f: for a diagonal P the single product is the binary32
    product of the binary32-rounded operands."""
    rng = np.random.default_rng(12)
    n = 50
    pv = rng.standard_normal(n).astype(np.float32).astype(np.float64)
    d = rng.uniform(0.5, 2.0, n)
    b = rng.standard_normal(n)
    x0 = O.x0(np.arange(n + 1), np.arange(n), pv, d, b, "fp32")
    expect = (pv.astype(np.float32) * (d * b).astype(np.float32)).astype(np.float64)
    assert np.array_equal(x0, expect)


# ---------------------------------------------------------------------------
# working precision single (the precision sets of Tables 4 and 5)
# ---------------------------------------------------------------------------

def _f32(a):
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


def test_fp32_gmres_step_is_the_krylov_least_squares_minimiser():
    """u = single: after k iterations (tau = 0) the correction is the Krylov
    least-squares minimiser of the binary32 data (A and b rounded to binary32,
    x0 and r0 stored in binary32, r0 evaluated in binary64), up to binary32
    rounding of the Arnoldi process."""
    rng = np.random.default_rng(21)
    n = 8
    Ad = _f32(_random_dd(n, rng, density=0.6, dom=0.4))
    A = _csr(Ad)
    b = _f32(rng.standard_normal(n))
    pp, pc, pv, d = np.arange(n + 1), np.arange(n), np.ones(n), np.ones(n)
    x0 = _f32(O.x0(pp, pc, pv, d, b, "fp32"))
    r0 = _f32(b - Ad @ x0)
    for k in range(1, 6):
        res = O.gmres_ir(A, pp, pc, pv, d, "fp32", b, 0.0, 1, k, 0.0, "mgs", "fp32")
        assert res.its == [k]
        assert np.array_equal(_f32(res.x), res.x)           # x is stored in binary32
        K = np.column_stack([np.linalg.matrix_power(Ad, i) @ r0 for i in range(k)])
        Q, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(Ad @ Q, r0, rcond=None)
        dexp = Q @ y
        assert np.abs((res.x - x0) - dexp).max() <= 2e-5 * np.abs(dexp).max() + 4 * 2.0 ** -24 * np.abs(x0).max()


def test_fp32_exact_preconditioner_takes_one_iteration_per_step():
    """P = A^-1 rounded to binary32 (u_f = single = u): every refinement step
    takes one GMRES iteration (the 1(1)-type rows of Table 5), and the
    refinement reaches the binary32 limiting accuracy."""
    w = W.s0_matrix(5)
    Ad = _dense(w.A)
    S = sp.csr_matrix(_f32(np.linalg.inv(Ad)))
    S.sort_indices()
    res = O.gmres_ir(w.A, S.indptr, S.indices, S.data, np.ones(w.n), "fp32", w.b, 1e-4, 10, 50, W.TOL_IR32,
                     "mgs", "fp32")
    assert all(k == 1 for k in res.its), res.its
    assert O.ferr(res.x, w.x_true) <= 2.0 ** -22


def test_fp32_limiting_accuracy_and_half_vs_single():
    """Theorem 1 with u = single, u_r = double: the forward error reaches the
    order of u (here x_true is a binary32 vector); SPAI in half and in single
    give near-identical nnz(P) and iteration totals (Tables 4 and 5)."""
    w = W.s0_matrix(6)
    n, ir = w.n, w.ir
    assert ir.u == "fp32" and ir.tau == 1e-4
    tot = {}
    for uf in ("fp16", "fp32"):
        R = O.spai(w.A, None, 0.3, -(-n // 8), 8, 63, uf)
        pp, pc, pv = R.P_csr(n)
        res = O.gmres_ir(w.A, pp, pc, pv, R.d, uf, w.b, ir.tau, ir.imax, ir.maxit, ir.tol_ir, "mgs", "fp32")
        assert res.status & ~O.IR_STAGNATED == 0
        assert O.ferr(res.x, w.x_true) <= 2.0 ** -20
        tot[uf] = (int(pp[-1]), sum(res.its))
    assert abs(tot["fp16"][0] - tot["fp32"][0]) <= 0.05 * tot["fp32"][0]
    assert abs(tot["fp16"][1] - tot["fp32"][1]) <= 0.25 * tot["fp32"][1] + 2
    with pytest.raises(ValueError):
        O.gmres_ir(w.A, pp, pc, pv, R.d, "fp32", w.b, ir.tau, 1, 5, ir.tol_ir, "dcgs2", "fp32")


# ---------------------------------------------------------------------------
# right preconditioning (GMRES on A P y = r, the paper's future-work variant)
# ---------------------------------------------------------------------------

def test_right_spai_columns_meet_eps_on_A():
    """The right build is Algorithm 1 on A itself: with P = D M, column k of
    A P - I is A D m_k - e_k, whose norm is the column residual the build
    reports and tests against eps."""
    w = W.convdiff_small(12)
    n = w.n
    R, pp, pc, pv, d = O.spai_right(w.A, None, 0.4, -(-n // 8), 8, 20, "fp64")
    P = sp.csr_matrix((pv, pc, pp), shape=(n, n)).toarray() * d[:, None]
    E = _dense(w.A) @ P - np.eye(n)
    colres = np.linalg.norm(E, axis=0)
    assert np.allclose(colres, R.res, rtol=1e-9, atol=1e-12)
    ok = (R.flags & O.FLAG_EPS) == 0
    assert ok.any() and np.all(colres[ok] <= 0.4 * (1 + 1e-12))


def test_right_gmres_step_is_the_krylov_least_squares_minimiser():
    """Right preconditioning: after k iterations (tau = 0) the correction is
    d = P y with y = argmin over K_k(A P, r0) of ||r0 - A P y||_2."""
    rng = np.random.default_rng(31)
    n = 8
    Ad = _random_dd(n, rng, density=0.6, dom=0.4)
    A = _csr(Ad)
    b = rng.standard_normal(n)
    R, pp, pc, pv, d = O.spai_right(A, None, 0.6, 0, 8, 8, "fp64")      # a diagonal P
    P = sp.csr_matrix((pv, pc, pp), shape=(n, n)).toarray() * d[:, None]
    x0 = O.x0_right(pp, pc, pv, d, b, "fp64")
    r0 = b - Ad @ x0
    AP = Ad @ P
    for ortho in ("mgs", "dcgs2"):
        for k in range(1, 6):
            res = O.gmres_ir(A, pp, pc, pv, d, "fp64", b, 0.0, 1, k, 0.0, ortho, side="right")
            assert res.its == [k]
            K = np.column_stack([np.linalg.matrix_power(AP, i) @ r0 for i in range(k)])
            Q, _ = np.linalg.qr(K)
            y, *_ = np.linalg.lstsq(AP @ Q, r0, rcond=None)
            dexp = P @ (Q @ y)
            assert np.abs((res.x - x0) - dexp).max() <= 1e-9 * np.abs(dexp).max()


def test_right_exact_preconditioner_takes_one_iteration_per_step():
    w = W.convdiff_small(10)
    S = sp.csr_matrix(np.linalg.inv(_dense(w.A)))
    S.sort_indices()
    res = O.gmres_ir(w.A, S.indptr, S.indices, S.data, np.ones(w.n), "fp64", w.b, 1e-8, 10, 50, W.TOL_IR,
                     side="right")
    assert all(k == 1 for k in res.its)
    assert O.ferr(res.x, w.x_true) <= 1e-15


# ---------------------------------------------------------------------------
# applying P = M^T D and the initial solve with a non-diagonal P and a
# non-constant scaling (where D applied on the wrong side of M^T would show)
# ---------------------------------------------------------------------------

_U = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8, "fp32": 2.0 ** -24, "fp64": 2.0 ** -53}


def _nondiagonal_spai(uf):
    """A fixed-pattern SPAI of the 12x12 convection-diffusion matrix on pattern(A):
    rows of 3-5 entries, values rounded to u_f by the build."""
    w = W.convdiff_adaptive(12)
    R = O.spai(w.A, W.pattern_of(w.A), 0.3, 0, 8, 20, uf)
    pp, pc, pv = R.P_csr(w.n)
    assert np.diff(pp).max() >= 4
    return w, pp, pc, pv


def _wide_vector(rng, n):
    return rng.standard_normal(n) * 10.0 ** rng.uniform(-3, 3, n)


def test_apply_P_is_Mt_times_D_for_a_nondiagonal_P():
    """Section 4 / Algorithm 3: P = M^T D, so y = P w = M^T (D w); checked against
    scipy's (M^T diag(d)) w with d non-constant, within the FP64 rounding of the
    row sums (D (M^T w) differs at the O(1) level)."""
    w, pp, pc, pv = _nondiagonal_spai("fp64")
    rng = np.random.default_rng(41)
    n = w.n
    d = rng.uniform(0.25, 4.0, n)
    MT = sp.csr_matrix((pv, pc, pp), shape=(n, n))
    q = np.diff(pp)
    for _ in range(5):
        v = _wide_vector(rng, n)
        y = O.apply_P(pp, pc, pv, d, v)
        ref = (MT @ sp.diags(d)) @ v
        scale = abs(MT) @ np.abs(d * v)
        assert np.all(np.abs(y - ref) <= (q + 2) * _U["fp64"] * scale)
        wrong = d * (MT @ v)
        assert np.abs(wrong - ref).max() > 1e-3 * np.abs(ref).max()


@pytest.mark.parametrize("uf", ["fp64", "fp32", "fp16", "bf16"])
def test_x0_is_Mt_D_b_in_uf_for_a_nondiagonal_P(uf):
    """Algorithm 3, initial solve: x0 = P b in u_f = M^T (D b) with D b rounded to
    u_f and the row sums in the arithmetic precision of u_f (binary32 for
    FP16/BF16).  Upper bound: the u_f rounding of D b plus the sum's rounding;
    lower bound (16-bit formats): the largest error reaches the order of u_f,
    so the storage rounding of D b is really there."""
    w, pp, pc, pv = _nondiagonal_spai(uf)
    rng = np.random.default_rng(42)
    n = w.n
    d = rng.uniform(0.25, 4.0, n)
    MT = sp.csr_matrix((pv, pc, pp), shape=(n, n))
    q = np.diff(pp)
    arith = _U["fp64"] if uf == "fp64" else _U["fp32"]
    store = 0.0 if uf in ("fp64", "fp32") else _U[uf]
    worst = 0.0
    for _ in range(8):
        b = _wide_vector(rng, n)
        x0 = O.x0(pp, pc, pv, d, b, uf)
        ref = MT @ (d * b)
        scale = abs(MT) @ np.abs(d * b)
        err = np.abs(x0 - ref) / scale
        assert np.all(err <= 1.01 * (store + (q + 3) * arith)), (uf, err.max())
        worst = max(worst, err.max())
        wrong = d * (MT @ b)
        assert np.abs(wrong - ref).max() > 1e-3 * np.abs(ref).max()
    if store:
        assert worst >= 0.25 * store, (uf, worst)


def test_gmres_step_minimiser_with_a_nondiagonal_P():
    """The Krylov least-squares pin of GMRES with P = M^T D from a pattern(A)
    SPAI of a random 8x8 matrix (non-diagonal P, non-constant d): z = P r0 and
    the operator P A use D on the right of M^T."""
    rng = np.random.default_rng(43)
    n = 8
    Ad = _random_dd(n, rng, density=0.6, dom=0.4)
    A = _csr(Ad)
    b = rng.standard_normal(n)
    R = O.spai(A, W.pattern_of(A), 0.6, 0, 8, 8, "fp64")
    assert not np.allclose(R.d, R.d[0])
    pp, pc, pv = R.P_csr(n)
    assert pp[-1] > n                                   # not diagonal
    P = (sp.csr_matrix((pv, pc, pp), shape=(n, n)) @ sp.diags(R.d)).toarray()
    for ortho in ("mgs", "cgs2", "dcgs2"):
        for k in range(1, 6):
            res = O.gmres_ir(A, pp, pc, pv, R.d, "fp64", b, 0.0, 1, k, 0.0, ortho)
            assert res.its == [k]
            x0 = P @ b
            r0 = b - Ad @ x0
            z = P @ r0
            PA = P @ Ad
            K = np.column_stack([np.linalg.matrix_power(PA, i) @ z for i in range(k)])
            Q, _ = np.linalg.qr(K)
            y, *_ = np.linalg.lstsq(PA @ Q, z, rcond=None)
            dexp = Q @ y
            assert np.abs((res.x - x0) - dexp).max() <= 1e-9 * np.abs(dexp).max(), (ortho, k)


def _to_uf(x, uf):
    """Round binary64 values to u_f through binary32 (numpy / torch conversions)."""
    x32 = np.asarray(x, np.float64).astype(np.float32)
    if uf == "fp16":
        return x32.astype(np.float16).astype(np.float64)
    if uf == "bf16":
        torch = pytest.importorskip("torch")
        return torch.tensor(x32).to(torch.bfloat16).to(torch.float64).numpy()
    return x32.astype(np.float64) if uf == "fp32" else np.asarray(x, np.float64)


@pytest.mark.parametrize("uf", ["fp64", "fp32", "fp16", "bf16"])
def test_x0_right_is_D_M_fl_b(uf):
    """Right preconditioning: x0 = P b in u_f with P = D M, i.e. row i of M applied
    to b rounded to u_f, times d_i rounded to u_f.  The two storage points are
    checked apart: with d on the u_f grid only b's rounding shows (it reaches the
    order of u_f for the 16-bit formats), with b on the grid only d's rounding
    (x0 then equals fl(d) (M b) up to the binary32 sum)."""
    w = W.convdiff_adaptive(12)
    n = w.n
    _, pp, pc, pv, d = O.spai_right(w.A, W.pattern_of(w.A), 0.3, 0, 8, 20, uf)
    assert np.diff(pp).max() >= 4 and not np.allclose(d, d[0])
    M = sp.csr_matrix((pv, pc, pp), shape=(n, n))
    q = np.diff(pp)
    arith = _U["fp64"] if uf == "fp64" else _U["fp32"]
    store = 0.0 if uf in ("fp64", "fp32") else _U[uf]
    rng = np.random.default_rng(44)
    worst_b = worst_d = 0.0
    for _ in range(8):
        b = _wide_vector(rng, n)
        dg = _to_uf(rng.uniform(0.25, 4.0, n), uf)          # d on the u_f grid
        x0 = O.x0_right(pp, pc, pv, dg, b, uf)
        ref = dg * (M @ b)
        scale = dg * (abs(M) @ np.abs(b))
        err = np.abs(x0 - ref) / scale
        assert np.all(err <= 1.01 * (store + (q + 4) * arith)), (uf, err.max())
        worst_b = max(worst_b, err.max())
        wrong = M @ (dg * b)
        assert np.abs(wrong - ref).max() > 1e-3 * np.abs(ref).max()

        bg = _to_uf(_wide_vector(rng, n), uf)               # b on the u_f grid
        x0 = O.x0_right(pp, pc, pv, d, bg, uf)
        scale = np.abs(d) * (abs(M) @ np.abs(bg))
        assert np.all(np.abs(x0 - _to_uf(d, uf) * (M @ bg)) <= 1.01 * (q + 4) * arith * scale)
        worst_d = max(worst_d, (np.abs(x0 - d * (M @ bg)) / scale).max())
    if store:
        assert worst_b >= 0.25 * store and worst_d >= 0.25 * store, (uf, worst_b, worst_d)


def _reduced_matrix(A, d, J):
    I = sorted({int(i) for j in J for i in A.col[A.rowptr[j]:A.rowptr[j + 1]]})
    pos = {i: t for t, i in enumerate(I)}
    Ab = np.zeros((len(I), len(J)))
    for c, j in enumerate(J):
        for t in range(A.rowptr[j], A.rowptr[j + 1]):
            Ab[pos[int(A.col[t])], c] = d[j] * A.val[t]
    return Ab, pos


@pytest.mark.parametrize("uf", ["fp32", "fp16", "bf16"])
def test_low_precision_columns_within_the_ls_perturbation_bound(uf):
    """Fixed pattern(A^2) columns of the 6^3 anisotropic system in u_f against the
    FP64 least-squares definition (eq. redprob): the relative difference stays
    within max(tol, 4 x Higham's LS perturbation bound kappa u_f +
    kappa^2 u_f ||s|| / (||A-bar|| ||m||)), tol = 1e-5 (FP32) or 2e-2 (16-bit);
    and the largest difference reaches the order of u_f, so the storage
    roundings of the QR are really there."""
    w = W.aniso_fixed(6, uf)
    s = w.spai
    R = O.spai(w.A, w.pattern, s.eps, s.alpha, s.beta, s.maxfill, uf)
    u = _U[uf]
    tol = 1e-5 if uf == "fp32" else 2e-2
    worst = 0.0
    for k in range(w.n):
        L = R.length[k]
        J = R.J[k, :L]
        mls, _ = O.ls_column(w.A, R.d, k, J)
        Ab, pos = _reduced_matrix(w.A, R.d, J)
        e = np.zeros(Ab.shape[0])
        e[pos[k]] = 1.0
        kap = np.linalg.cond(Ab)
        sres = np.linalg.norm(Ab @ mls - e)
        bound = kap * u + kap ** 2 * u * sres / (np.linalg.norm(Ab, 2) * np.linalg.norm(mls))
        rel = np.linalg.norm(R.m[k, :L] - mls) / np.linalg.norm(mls)
        assert rel <= max(tol, 4 * bound), (uf, k, rel, bound)
        worst = max(worst, rel)
    assert worst >= 0.5 * u, (uf, worst)


def _grid_matrix(n, rng, bits=8):
    """Random sparse diagonally dominant matrix whose entries have at most `bits`
    significant bits (inside the FP16 normal range) and whose diagonal is a power
    of two and the largest entry of its row: the scaling d_i is then a power of
    two and every entry of B = A^T D is a binary16 and a bfloat16 value."""
    M = rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.25)
    np.fill_diagonal(M, 0.0)
    M = np.where(M != 0, np.sign(M) * np.maximum(np.abs(M), 2.0 ** -6), 0.0)
    e = np.floor(np.log2(np.abs(np.where(M != 0, M, 1.0))))
    M = np.where(M != 0, np.round(M * 2.0 ** (bits - 1 - e)) * 2.0 ** (e - bits + 1), 0.0)
    np.fill_diagonal(M, 2.0 ** np.ceil(np.log2(1.5 * np.abs(M).sum(1) + 1.0)))
    return M


@pytest.mark.parametrize("uf", ["fp16", "bf16"])
def test_gathered_entries_are_rounded_to_uf(uf):
    """Storage point 'A-bar rounded to u_f' (Section 3.1's u_f build): a matrix
    whose scaled entries are u_f values and the same matrix with every
    off-diagonal entry moved by a relative 2^-14 (well inside half a u_f ulp)
    gather the same u_f A-bar, so Algorithm 1 gives bit-identical columns, fixed
    and adaptive; without that rounding they differ."""
    rng = np.random.default_rng(45)
    n = 40
    Ad = _grid_matrix(n, rng)
    off = ~np.eye(n, dtype=bool) & (Ad != 0)
    Ap = Ad.copy()
    Ap[off] *= 1.0 + np.where(rng.random(off.sum()) < 0.5, -1.0, 1.0) * 2.0 ** -14
    A, A2 = _csr(Ad), _csr(Ap)
    for pattern, alpha in ((W.pattern_of(A), 0), (None, 5)):
        R1 = O.spai(A, pattern, 0.2, alpha, 8, 20, uf)
        R2 = O.spai(A2, pattern, 0.2, alpha, 8, 20, uf)
        assert np.array_equal(R1.d, R2.d)
        assert np.array_equal(R1.J, R2.J) and np.array_equal(R1.m, R2.m)
        assert np.array_equal(_to_uf(R1.m, uf), R1.m)        # m-bar is stored in u_f
    R64 = O.spai(A, None, 0.2, 5, 8, 20, "fp64")
    R64p = O.spai(A2, None, 0.2, 5, 8, 20, "fp64")
    assert not np.array_equal(R64.m, R64p.m)                  # the perturbation is seen in FP64


def _overflow_system(n=24):
    """Upper bidiagonal A = I - 2 N: (A^-1)_kj = 2^(j-k), so the SPAI of B = A^T D on
    the pattern of A^-1 has entries up to ~2^(n-1), far beyond the FP16 range
    (65504), although every entry of B (0.5, -1) is exact in FP16."""
    A = np.eye(n) + np.diag(-2.0 * np.ones(n - 1), 1)
    Ai = np.linalg.inv(A)
    ptr, idx = [0], []
    for k in range(n):
        idx += list(np.nonzero(Ai[k])[0])
        ptr.append(len(idx))
    pat = W.Pattern(n, np.array(ptr, np.int32), np.array(idx, np.int32))
    return A, _csr(A), pat


def test_fp16_overflow_columns_are_recomputed_in_fp32():
    """Overflow policy of the 16-bit build (Section 4's scaling keeps the half
    precision computations in range only where the reduced problems allow it):
    exactly the columns whose values exceed the FP16 range are recomputed, and
    they then equal the FP32 build of the same column bit for bit; the others
    keep their FP16 values; the solve with the resulting P converges."""
    Ad, A, pat = _overflow_system()
    n = A.n
    R16 = O.spai(A, pat, 0.5, 0, 8, 63, "fp16")
    R32 = O.spai(A, pat, 0.5, 0, 8, 63, "fp32")
    fb = (R16.flags & O.FLAG_FALLBACK) != 0
    big = np.abs(R32.m).max(axis=1) > 65504.0
    assert fb.sum() >= 4 and np.array_equal(fb, big)
    assert not np.any(R16.flags & O.FLAG_NONFINITE)
    assert np.array_equal(R16.m[fb], R32.m[fb]) and np.array_equal(R16.J[fb], R32.J[fb])
    assert np.all(np.isfinite(R16.m))
    assert np.array_equal(_to_uf(R16.m[~fb], "fp16"), R16.m[~fb])       # FP16 values kept
    R16b = O.spai(A, pat, 0.5, 0, 8, 63, "bf16")                          # BF16 has FP32's range
    assert not np.any(R16b.flags & O.FLAG_FALLBACK)
    x_true = np.linspace(-1.0, 1.0, n)
    b = Ad @ x_true
    pp, pc, pv = R16.P_csr(n)
    res = O.gmres_ir(A, pp, pc, pv, R16.d, "fp16", b, 1e-8, 10, n, W.TOL_IR)
    assert res.status & ~O.IR_STAGNATED == 0 and O.ferr(res.x, x_true) <= 1e-12


def test_fp32_refinement_restarted_from_an_iterate_repeats_its_steps():
    """Refinement is a chain in x: started from the iterate x_i of a run (warm
    start), one step reproduces that run's step i (its GMRES count and x_{i+1},
    bit for bit), and started from the exact solution no step is taken (P r = 0,
    Algorithm 3's residual is exactly zero)."""
    w = W.s0_matrix(5)
    n, ir = w.n, w.ir
    R = O.spai(w.A, None, 0.3, -(-n // 8), 8, 63, "fp16")
    pp, pc, pv = R.P_csr(n)
    full = O.gmres_ir(w.A, pp, pc, pv, R.d, "fp16", w.b, ir.tau, ir.imax, ir.maxit, ir.tol_ir, "mgs", "fp32")
    assert len(full.its) >= 2 and full.xhist.shape == (len(full.its) + 1, n)
    assert np.array_equal(full.xhist[-1], full.x)
    assert np.all((full.gest <= ir.tau) & (full.gprev > ir.tau))
    for i, k in enumerate(full.its):
        one = O.gmres_ir(w.A, pp, pc, pv, R.d, "fp16", w.b, ir.tau, 1, ir.maxit, ir.tol_ir, "mgs", "fp32",
                         x_init=full.xhist[i])
        assert one.its == [k] and np.array_equal(one.x, full.xhist[i + 1]), i
    exact = O.gmres_ir(w.A, pp, pc, pv, R.d, "fp16", w.b, ir.tau, 3, ir.maxit, ir.tol_ir, "mgs", "fp32",
                       x_init=w.x_true)
    assert exact.its == [] and np.array_equal(exact.x, w.x_true)


def test_flop_count_of_a_fixed_pattern_build():
    """The algorithmic flop count of a fixed-pattern build (one m x p solve per
    column, Section 2.2's cost cubic in the entries per column) equals the
    formula evaluated on shadow sizes counted independently: |I_k| = the
    number of columns of row k of pattern(P) x pattern(A)."""
    w = W.aniso_fixed(6, "fp32")
    s = w.spai
    R = O.spai(w.A, w.pattern, s.eps, s.alpha, s.beta, s.maxfill, "fp32")
    n = w.n
    Ap = sp.csr_matrix((np.ones(w.A.nnz), w.A.col, w.A.rowptr), shape=(n, n))
    Pp = sp.csr_matrix((np.ones(w.pattern.nnz), w.pattern.idx, w.pattern.ptr), shape=(n, n))
    m = np.diff((Pp @ Ap).indptr).astype(float)
    p = np.diff(w.pattern.ptr).astype(float)
    assert np.array_equal(R.nI, m.astype(np.int32)) and np.array_equal(R.length, p.astype(np.int32))
    assert np.allclose(R.flops, 2 * m * p * p - 2 * p ** 3 / 3 + 4 * m * p + p * p, rtol=1e-15)
    Ra = O.spai(w.A, None, 0.3, 5, 8, 20, "fp32")              # adaptive: one term per solve
    assert np.all(Ra.flops >= 2 * Ra.nI * Ra.length ** 2 - 2 * Ra.length ** 3 / 3)
    assert np.all((Ra.steps > 0) <= (Ra.flops > 2 * Ra.nI * Ra.length ** 2))
