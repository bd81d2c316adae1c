"""The paper's accuracy experiment on its unsymmetric model problem (TP2 of the
table of test problems: 1000 x 1000 5-point stencil with the entries above
the diagonal -1 + 1e-3, normalised to ||A||_2 = 1, b = A 1/sqrt(N), x_0 = 0,
no preconditioner), run on the GPU and checked against what Section 4
reports for it (orders of magnitude only: the paper ran on 120 MPI ranks
with other reduction orders):

* classic BiCGStab reaches a ~1e-13 relative true residual in ~600 iterations;
* p-BiCGStab without replacement stalls: its best true residual is ~1e-10,
  orders of magnitude above classic, although its recursive residual keeps
  falling (the residual gap of Section 3);
* p-BiCGStab with replacement every 100 iterations reaches ~1e-13 again;
* the automated strategy (Section 3.6) reaches it with about ten
  replacements (here: see the test; the schedule is rounding-sensitive).

The oracle on the same problem (NumPy, FP64): classic 566 iterations, true
residual 1.6e-13; replacement every 100: 823 iterations, 5 replacements,
4.3e-14; without replacement it breaks down (rho' = 0) after 2716
iterations with a true residual of 3.6e-4.
"""

import numpy as np
import pytest
import torch

from gpu_util import dev, history_buffer, host, split_history
from workloads import tp2_unsymmetric

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp2():
    return tp2_unsymmetric(1000)


@pytest.fixture(scope="module")
def solver(tp2):
    from paper_1809_01948_amd.solver import Solver
    S = Solver.from_problem(tp2, form="stencil", precond="none")
    yield S
    S.close()


def test_tp2_classic_reaches_1e13(solver, tp2):
    x, st = solver.solve(dev(tp2.b), tol=1e-13, maxit=3000, method="classic")
    print("classic", st, flush=True)
    assert st["rel_res_true"] <= 3e-13
    assert 400 <= st["iterations"] <= 900


def test_tp2_pipelined_attainable_accuracy(solver, tp2):
    """Without replacement: the best true residual along the run stays far
    above classic's, while the recursive residual goes far below it.  Solves
    are bitwise repeatable, so stopping the same run after k iterations
    samples its true residual ||b - A x_k|| exactly."""
    b = dev(tp2.b)
    hist = history_buffer(1500)
    x, st = solver.solve(b, tol=0.0, maxit=1500, history=hist)
    rn, _, _, _ = split_history(hist, st["iterations"])
    rec_min = rn.min() / np.linalg.norm(tp2.b)
    true = []
    for k in range(300, st["iterations"] + 1, 50):
        _, sk = solver.solve(b, tol=0.0, maxit=k)
        true.append(sk["rel_res_true"])
    best = min(true)
    print(f"p-BiCGStab: {st['status_name']} after {st['iterations']}, best true {best:.2e}, "
          f"min recursive {rec_min:.2e}", flush=True)
    # classic reaches ~1.5e-13 on this problem (previous test); the paper ~1e-10
    assert 1e-12 <= best <= 1e-8


def test_tp2_periodic_replacement_restores_accuracy(solver, tp2):
    x, st = solver.solve(dev(tp2.b), tol=1e-13, maxit=3000, rr_period=100)
    print("P=100", st, flush=True)
    assert st["status"] == 0 and st["rel_res_true"] <= 1e-13
    assert 1 <= st["replacements"] <= 15
    assert st["iterations"] <= 1500


def test_tp2_automated_replacement(solver, tp2):
    """Automated replacement (Section 3.6, worst-case bound eq:DDr_bound and
    eq:criterion) on TP2.  The paper reports ten replacements, all early, and
    an attainable accuracy near classic's (~1e-13).  What happens after the
    last replacement is as rounding-sensitive as the iterates: the bound's
    restart value after a replacement, ((mu sqrt(N) + 1) ||A|| ||x|| + ||b||)
    eps, exceeds tau ||r|| once ||r|| < 7e-3 ||b||, so the criterion cannot
    fire later, and whether the gap then stays small depends on the last bits
    of the run (the same problem with b perturbed by 1e-15 relative reaches
    1e-11 in one run and stalls at 1e-7 in another).  Checked on three such
    draws: a few replacements, all within the first 300 iterations; every
    draw keeps a best true residual <= 1e-6 (far below the 1e-3 level at which
    p-BiCGStab's gap makes it stall without any replacement); and at least
    one reaches 1e-10, p-BiCGStab's attainable accuracy without replacement.
    Not reproduced: the paper's ~1e-13 (the design notes list the oracle's
    outcomes over grid sizes and both readings of the bound)."""
    bests = []
    for j in range(3):
        b = dev(tp2.b * (1.0 + j * 1e-15))
        _, s300 = solver.solve(b, tol=0.0, maxit=300, rr_auto="bound")
        _, s1000 = solver.solve(b, tol=0.0, maxit=1000, rr_auto="bound")
        assert 3 <= s300["replacements"] <= 20
        assert s1000["replacements"] == s300["replacements"]
        true = []
        for k in range(100, 1001, 100):
            _, sk = solver.solve(b, tol=0.0, maxit=k, rr_auto="bound")
            true.append(sk["rel_res_true"])
            if sk["iterations"] < k:
                break
        print(f"draw {j}: {s300['replacements']} replacements, true residual every 100 "
              f"iterations {['%.1e' % t for t in true]}", flush=True)
        bests.append(min(true))
    assert max(bests) <= 1e-6
    assert min(bests) <= 1e-10


@pytest.mark.parametrize("variant", ["estimate", "products-estimate"])
def test_tp2_automated_estimate_random_shadow(solver, tp2, variant):
    """The automated strategy with the square-root estimate of the bound
    (Section 3.6), in either reading, and a random fixed shadow vector (an
    option outside the paper), on two shadow vectors and two rounding-
    perturbed right-hand sides.

    * The criterion alone (no stopping test: the same run sampled every 100
      iterations up to 1,500) keeps the true residual down: best <= 5e-11
      (1e-11 with the nested reading) and <= 1e-8 after 1,500 iterations (or
      where the run stops at a rho' = 0 breakdown once its recursive residual
      has reached the rounding level), where p-BiCGStab without replacement
      has grown to ~1e-2 (Section 4.5:
      the automated strategy's accuracy is comparable to classic's, 1.4e-13
      here; measured 1.2e-13 to 3e-12 with the nested reading).
    * A solve to 1e-13 converges: the stopping test's confirm-and-replace
      (at most three replacements) closes the rest."""
    for seed in (56, 57):
        rh = dev(np.random.default_rng(seed).standard_normal(tp2.n))
        for j in range(2):
            b = dev(tp2.b * (1.0 + j * 1e-15))
            traj = []
            for k in range(300, 1501, 100):
                _, st = solver.solve(b, tol=0.0, maxit=k, rr_auto=variant, rhat=rh)
                traj.append(st["rel_res_true"])
                if st["iterations"] < k:    # a rho' = 0 stop at the noise floor ends it
                    break
            _, st = solver.solve(b, tol=1e-13, maxit=3000, rr_auto=variant, rhat=rh)
            print(f"{variant} shadow {seed} draw {j}: criterion alone best {min(traj):.2e}, "
                  f"at the end {traj[-1]:.2e}; to 1e-13: {st['status_name']} "
                  f"{st['iterations']} iterations, {st['replacements']} replacements, "
                  f"true {st['rel_res_true']:.2e}", flush=True)
            assert min(traj) <= (1e-11 if variant == "estimate" else 5e-11)
            assert traj[-1] <= 1e-8
            assert st["status"] == 0 and st["rel_res_true"] <= 1e-13
            assert 5 <= st["replacements"] <= 150 and st["iterations"] <= 1500


@pytest.mark.parametrize("variant", ["estimate", "products-estimate"])
def test_tp2_automated_estimate_nv_refresh(solver, tp2, variant):
    """Section 4.5's TP2 result with the paper's shadow residual r_0 when
    every replacement also refreshes n = M^-1 z and v = A n from the
    replaced z (pbcg_opts.rr_nv, an option outside the paper): the automated
    criterion with the square-root estimate alone keeps the true residual at
    the classic level (best ~1e-13; without the refresh the same runs reach
    3e-9 and 5e-6), and a solve to 1e-13 converges with a handful of
    replacements (the paper: 10)."""
    b = dev(tp2.b)
    traj = []
    for k in range(300, 1501, 100):
        _, st = solver.solve(b, tol=0.0, maxit=k, rr_auto=variant, rr_nv=True)
        traj.append(st["rel_res_true"])
        if st["iterations"] < k:
            break
    _, st = solver.solve(b, tol=1e-13, maxit=3000, rr_auto=variant, rr_nv=True)
    print(f"{variant} + refresh: criterion alone best {min(traj):.2e}; to 1e-13: "
          f"{st['status_name']} {st['iterations']} iterations, {st['replacements']} "
          f"replacements, true {st['rel_res_true']:.2e}", flush=True)
    assert min(traj) <= 5e-13
    assert st["status"] == 0 and st["rel_res_true"] <= 1e-13
    assert 3 <= st["replacements"] <= 50 and st["iterations"] <= 1500


# -----------------------------------------------------------------------------
# TP3: the indefinite Helmholtz problem of Table tab:specs (500 x 500, shift
# 5e-4, ||A||_2 = 1, b = A 1/sqrt(N), no preconditioner, as in the timed runs
# of Section 4.1).  Section 4.6 reports (120 ranks): classic ~1e-8 after ~4000
# iterations; p-BiCGStab stuck near 1e-4 early on, 8e-5 after ~4000 and
# ~1e-9 only after ~7000; with replacement every 200 ~1e-8 after ~4000.
# -----------------------------------------------------------------------------

@pytest.fixture(scope="module")
def tp3():
    from workloads import tp3_helmholtz
    return tp3_helmholtz(500)


def _true_after(S, b, k, **kw):
    """True residual of the same (bitwise repeatable) run stopped after k
    iterations."""
    _, st = S.solve(b, tol=0.0, maxit=k, **kw)
    return st["iterations"], st["rel_res_true"]


def test_tp3_accuracy_orders_of_magnitude(tp3):
    from paper_1809_01948_amd.solver import Solver
    S = Solver.from_problem(tp3, form="stencil", precond="none")
    b = dev(tp3.b)
    ks = range(500, 8001, 500)
    classic = [_true_after(S, b, k, method="classic") for k in ks]
    plain = [_true_after(S, b, k) for k in ks]
    rr = [_true_after(S, b, k, rr_period=200) for k in ks]
    print("classic", classic, "\np", plain, "\np-rr200", rr, flush=True)
    best = lambda run: min(r for _, r in run)
    # classic reaches the paper's accuracy (or better) within ~4000 iterations
    assert min(r for k, r in classic if k <= 4000) <= 1e-8
    # without replacement p-BiCGStab plateaus early (its residual after 1000
    # iterations is still at the 1e-4 level) and never gets near classic's
    # accuracy; past its best point the true residual grows again
    assert dict(plain)[1000] >= 1e-5
    assert best(plain) >= 10 * best(classic)
    assert plain[-1][1] >= 10 * best(plain)
    # with replacement every 200 it reaches classic's order of accuracy
    assert best(rr) <= 1e-8
    assert best(rr) <= 100 * best(classic)
    # with the n/v refresh on replacement (rr_nv, outside the paper) below
    # classic's best, and sooner (measured 1.8e-13 at 2,000 iterations)
    rrnv = [_true_after(S, b, k, rr_period=200, rr_nv=True) for k in ks if k <= 3000]
    print("p-rr200-nv", rrnv, flush=True)
    assert best(rrnv) <= best(classic)
    S.close()


# -----------------------------------------------------------------------------
# Section 3.3's error propagation matrices from a GPU run's recorded scalars
# -----------------------------------------------------------------------------

def test_propagation_norms_from_gpu_history():
    """The column maximum norms of the nine products of eq:all_error_matrices,
    built from the alpha, omega, beta a GPU solve records, equal those built
    from the oracle's scalars over the iterations where the two runs agree
    (the scalars agree to 1e-10 over the first 12 iterations; the oracle
    against itself with another summation order agrees that long), and they
    grow several orders of magnitude above one as Section 4.4 describes."""
    from oracle import Float64Ops, pipelined_bicgstab
    from paper_1809_01948_amd import diagnostics
    from paper_1809_01948_amd.solver import Solver
    from workloads import tp2_unsymmetric
    p = tp2_unsymmetric(200)
    A = p.scipy_csr()
    its = 150
    ref = pipelined_bicgstab(Float64Ops(A), p.b, tol=0.0, maxit=its)
    S = Solver.from_problem(p, form="stencil", precond="none")
    hist = history_buffer(its)
    x, st = S.solve(dev(p.b), tol=0.0, maxit=its, history=hist)
    assert st["iterations"] == its == ref.iterations
    rn, al, om, be = split_history(hist, its)
    k = 12
    gpu = diagnostics.column_max_norms(al[:k], om[:k], be[:k])
    ora = diagnostics.column_max_norms(ref.alpha[:k], ref.omega[:k], ref.beta[:k])
    for name in diagnostics.PRODUCTS:
        assert np.allclose(gpu[name], ora[name], rtol=1e-8, atol=0), name
    full = diagnostics.column_max_norms(al, om, be)
    top = max(float(np.max(full[name])) for name in diagnostics.PRODUCTS)
    assert top >= 1e3, top
    S.close()
