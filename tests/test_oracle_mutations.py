"""Plant plausible mistakes in the oracle (on the CPU, by monkeypatching) and check
that at least one pin catches each.  This is evidence that the pins constrain the
oracle rather than restate it."""
import numpy as np
import pytest

import tests.test_oracle_pins as pins
from oracle import wc4d_oracle as O


def _fails(fn, *a):
    try:
        fn(*a)
    except AssertionError:
        return True
    return False


def test_wrong_stencil_sign_is_caught(monkeypatch):
    monkeypatch.setattr(O, "advdiff_step", lambda x, c, r: (c + r) * np.roll(x, -1, 0) + (1 - c - 2 * r) * x + r * np.roll(x, 1, 0))
    assert _fails(pins.test_advdiff_fourier_multiplier, 0.5, 0.1)
    assert _fails(pins.test_advdiff_pure_upwind_courant_one_is_exact_shift)


def test_wrong_transpose_is_caught(monkeypatch):
    monkeypatch.setattr(O, "advdiff_step_T", lambda w, c, r: O.advdiff_step(w, c, r))
    assert _fails(pins.test_advdiff_transpose)
    assert _fails(pins.test_Linv_adjoint_dot_product, pins.tiny_advdiff)


def test_wrong_rk4_weight_is_caught(monkeypatch):
    def bad(x, F, dt):
        k1 = O.l96_rhs(x, F); k2 = O.l96_rhs(x + 0.5 * dt * k1, F)
        k3 = O.l96_rhs(x + 0.5 * dt * k2, F); k4 = O.l96_rhs(x + dt * k3, F)
        return x + (dt / 6.0) * (k1 + 2.0 * k2 + k3 + 2.0 * k4)
    monkeypatch.setattr(O, "l96_rk4_step", bad)
    assert _fails(pins.test_l96_rk4_fourth_order_against_reference_integrator)


def test_wrong_l96_sign_is_caught(monkeypatch):
    orig = O.l96_rhs
    monkeypatch.setattr(O, "l96_rhs", lambda x, F: orig(x, F) + 2 * np.roll(x, 2, 0) * np.roll(x, 1, 0))
    assert _fails(pins.test_l96_equilibrium_and_constant_forcing)


def test_tlm_missing_stage_term_is_caught(monkeypatch):
    orig = O._l96_jac
    monkeypatch.setattr(O, "_l96_jac", lambda y, d: orig(y, d) + d)
    assert _fails(pins.test_l96_tlm_matches_finite_differences)


def test_adjoint_dropped_term_is_caught(monkeypatch):
    orig = O._l96_jac_T
    # drop the -y_{j+1} a_{j+2} term of J^T a
    monkeypatch.setattr(O, "_l96_jac_T", lambda y, a: orig(y, a) + np.roll(y, -1, 0) * np.roll(a, -2, 0))
    assert _fails(pins.test_l96_adjoint_dot_product)


def test_missing_model_error_block_is_caught(monkeypatch):
    # sweep that forgets p_{i+1}
    def bad(prob, P):
        Pl = P.reshape(prob.N + 1, prob.n, -1)
        Xl = np.empty_like(Pl); Xl[0] = Pl[0]
        for i in range(prob.N):
            Xl[i + 1] = prob.M(i, Xl[i])
        return Xl.reshape(P.shape)
    monkeypatch.setattr(O, "apply_Linv", bad)
    assert _fails(pins.test_Linv_equals_block_formula, pins.tiny_advdiff)


def test_dsqrt_transposed_blocks_are_caught(monkeypatch):
    def bad(prob, X):
        Xl = X.reshape(prob.N + 1, prob.n, -1); Yl = np.empty_like(Xl)
        Yl[0] = prob.Qsqrt @ Xl[0]
        for i in range(1, prob.N + 1):
            Yl[i] = prob.Bsqrt @ Xl[i]
        return Yl.reshape(X.shape)
    monkeypatch.setattr(O, "apply_Dsqrt", bad)
    assert _fails(pins.test_A_equals_transformed_unpreconditioned_hessian, pins.tiny_advdiff)


def test_ritzit_without_square_root_is_caught(monkeypatch):
    orig = O.ritzit
    def bad(applyA, G, k):
        U, t = orig(applyA, G, k)
        return U, t * t
    monkeypatch.setitem(O.METHODS, "ritzit", bad)
    assert _fails(pins.test_full_sketch_recovers_exact_spectrum, "ritzit")


def test_lmp_wrong_exponent_is_caught(monkeypatch):
    monkeypatch.setattr(O, "lmp_dense_C", lambda U, th: np.eye(U.shape[0]) + U @ np.diag(1 / th - 1) @ U.T)
    assert _fails(pins.test_lmp_factor_identities)
    assert _fails(pins.test_exact_pair_lmp_spectrum_theorem)


def test_pcg_wrong_beta_is_caught(monkeypatch):
    orig = O.pcg
    def bad(applyA, b, x0=None, lmp=None, tol=1e-6, maxit=100, criterion=0):
        x = np.zeros_like(b); r = b.copy(); p = r.copy(); rr = r @ r
        hist = []
        for it in range(1, maxit + 1):
            Ap = applyA(p); a = rr / (p @ Ap); x = x + a * p; r = r - a * Ap
            rn = r @ r; p = r + (rr / rn) * p; rr = rn   # inverted beta
            hist.append(np.sqrt(rr) / np.linalg.norm(b))
            if hist[-1] <= tol:
                break
        return O.PCGResult(x, it, hist[-1] <= tol, hist[-1], hist[-1], 0.0, hist, hist, [0.0] * it, [], [])
    monkeypatch.setattr(O, "pcg", bad)
    assert _fails(pins.test_cg_finite_termination_on_three_distinct_eigenvalues)



def test_nystrom_without_square_is_caught(monkeypatch):
    orig = O.nystrom
    def bad(applyA, G, k):
        U, t = orig(applyA, G, k)
        return U, np.sqrt(t)
    monkeypatch.setitem(O.METHODS, "nystrom", bad)
    assert _fails(pins.test_full_sketch_recovers_exact_spectrum, "nystrom")


def test_nystrom_wrong_triangular_side_is_caught(monkeypatch):
    # F C^T = E1 in place of F C = E1 (Algorithm 4's triangular solve)
    import scipy.linalg as sla
    def bad(applyA, G, k):
        Z1 = O._orth(applyA(G))
        E1 = applyA(Z1)
        E2 = Z1.T @ E1
        C = np.linalg.cholesky(0.5 * (E2 + E2.T)).T
        F = sla.solve_triangular(C, E1.T, lower=False).T
        U2, sig, _ = np.linalg.svd(F, full_matrices=False)
        return U2[:, :k], sig[:k] ** 2
    monkeypatch.setitem(O.METHODS, "nystrom", bad)
    assert _fails(pins.test_full_sketch_recovers_exact_spectrum, "nystrom")
    assert _fails(pins.test_untruncated_outputs_equal_closed_forms, "nystrom")


def test_revd_keeping_smallest_pairs_is_caught(monkeypatch):
    def bad(applyA, G, k):
        Z1 = O._orth(applyA(G))
        K1 = Z1.T @ applyA(Z1)
        lam, W = np.linalg.eigh(0.5 * (K1 + K1.T))      # increasing order kept as is
        return Z1 @ W[:, :k], lam[:k]
    monkeypatch.setitem(O.METHODS, "revd", bad)
    assert _fails(pins.test_invariant_subspace_gives_exact_pairs, "revd")
    assert _fails(pins.test_ritz_values_bounds_and_orthonormality, "revd")


def test_ritzit_wrong_gram_side_is_caught(monkeypatch):
    # R^T R in place of R R^T: same eigenvalues, wrong eigenvectors (Algorithm 5)
    def bad(applyA, G, k):
        Z3, R3 = np.linalg.qr(applyA(O._orth(G)), mode="reduced")
        th2, W3 = O._eig_desc(R3.T @ R3)
        return Z3 @ W3[:, :k], np.sqrt(np.clip(th2[:k], 0.0, None))
    monkeypatch.setitem(O.METHODS, "ritzit", bad)
    assert _fails(pins.test_invariant_subspace_gives_exact_pairs, "ritzit")
    assert _fails(pins.test_untruncated_outputs_equal_closed_forms, "ritzit")


def test_observation_variance_in_place_of_its_inverse_is_caught(monkeypatch):
    def bad(prob, X):
        Xl = O._levels(prob, X)
        Zl = np.zeros_like(Xl)
        for i, idx, rdiag in prob.obs:
            np.add.at(Zl[i], idx, Xl[i][idx] * rdiag[:, None])
        return Zl.reshape(X.shape)
    monkeypatch.setattr(O, "apply_HtRinvH", bad)
    assert _fails(pins.test_A_equals_transformed_unpreconditioned_hessian, pins.tiny_advdiff)


def test_lmp_apply_with_projector_coefficients_is_caught(monkeypatch):
    # theta^{-1} - 1 (the projector P of eq. spectral_LMP) in place of theta^{-1/2} - 1
    def bad(U, th, X):
        d = 1.0 / th - 1.0
        return X + U @ ((d if X.ndim == 1 else d[:, None]) * (U.T @ X))
    monkeypatch.setattr(O, "lmp_apply", bad)
    assert _fails(pins.test_lmp_factor_identities)


def _split_pcg(c_in_r, c_in_p):
    """Algorithm 1 with switches that drop the preconditioner from the residual update
    (r_j = r_{j-1} - alpha A p) or from the direction (p = r + beta p)."""
    def pcg(applyA, b, x0=None, lmp=None, tol=1e-6, maxit=100, criterion=0):
        C = (lambda v: v) if lmp is None else (lambda v: O.lmp_apply(lmp[0], lmp[1], v))
        x = np.zeros_like(b)
        s = b.copy()
        r = C(s)
        p = C(r) if c_in_p else r.copy()
        r0 = np.linalg.norm(r)
        rr = r @ r
        ht, hp = [], []
        for it in range(1, maxit + 1):
            Ap = applyA(p)
            a = rr / (p @ Ap)
            x = x + a * p
            s = s - a * Ap
            r = r - a * (C(Ap) if c_in_r else Ap)
            rn = r @ r
            p = (C(r) if c_in_p else r) + (rn / rr) * p
            rr = rn
            ht.append(np.linalg.norm(s) / np.linalg.norm(b))
            hp.append(np.sqrt(rr) / r0)
            if (ht[-1] if criterion == O.RES_TRUE else hp[-1]) <= tol:
                break
        ok = (ht[-1] if criterion == O.RES_TRUE else hp[-1]) <= tol
        return O.PCGResult(x, it, ok, ht[-1], hp[-1], 0.0, ht, hp, [0.0] * it, [], [])
    return pcg


def test_split_pcg_rewrite_passes_the_pins(monkeypatch):
    # the switch-free rewrite is Algorithm 1 itself: it passes the pins the mutations fail
    monkeypatch.setattr(O, "pcg", _split_pcg(True, True))
    pins.test_full_rank_exact_lmp_converges_in_one_iteration()
    pins.test_pcg_precond_criterion_is_split_residual()


def test_pcg_residual_without_preconditioner_is_caught(monkeypatch):
    monkeypatch.setattr(O, "pcg", _split_pcg(False, True))
    assert _fails(pins.test_pcg_precond_criterion_is_split_residual)


def test_pcg_direction_without_second_preconditioner_is_caught(monkeypatch):
    monkeypatch.setattr(O, "pcg", _split_pcg(True, False))
    assert _fails(pins.test_full_rank_exact_lmp_converges_in_one_iteration)


# ------------------------------------------------------------ learned-sketch oracle
import tests.test_sketchnet_oracle as skpins  # noqa: E402
from oracle import sketchnet_oracle as SK  # noqa: E402


def test_sketchnet_wrong_tap_direction_is_caught(monkeypatch):
    orig = SK._conv
    monkeypatch.setattr(SK, "_conv", lambda W, b, A: orig(W[:, :, ::-1], b, A))
    assert _fails(skpins.test_conv_matches_fft_circular_correlation)
    assert _fails(skpins.test_conv_tap_direction_hand_example)


def test_sketchnet_dropped_tanh_derivative_is_caught(monkeypatch):
    orig = SK.backward

    def no_deriv(theta, acts, dG, round_fp16=True):
        params = SK._rounded(theta, acts[0].shape[1], round_fp16)
        T, _, n = acts[0].shape
        m = params[-1][0].shape[0]
        dH = dG.reshape(T, n, m).transpose(0, 2, 1)
        grads = []
        for l in range(len(params) - 1, -1, -1):
            W, b = params[l]
            A = acts[l]
            dW = np.zeros_like(W)
            for t in range(SK.KW):
                dW[:, :, t] = np.einsum("Ton,Tcn->oc", dH, np.roll(A, -(t - 2), axis=2))
            grads.append((dW, dH.sum(axis=(0, 2))))
            if l == 0:
                break
            dA = np.zeros_like(A)
            for t in range(SK.KW):
                dA += np.roll(np.einsum("oc,Ton->Tcn", W[:, :, t], dH), (t - 2), axis=2)
            dH = dA                      # missing (1 - A^2)
        grads.reverse()
        return np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    monkeypatch.setattr(SK, "backward", no_deriv)
    assert _fails(skpins.test_backward_matches_finite_differences)
    assert orig is not None


def test_capture_loss_gradient_sign_is_caught(monkeypatch):
    orig = SK.capture_loss

    def bad(applyA, G, U, theta):
        f, g = orig(applyA, G, U, theta)
        return f, -g
    monkeypatch.setattr(SK, "capture_loss", bad)
    assert _fails(skpins.test_capture_loss_through_operator_and_fd)


def test_adam_without_bias_correction_is_caught(monkeypatch):
    def bad(theta, g, mom, vel, step, lr, b1=0.9, b2=0.999, eps=1e-8):
        mom[:] = b1 * mom + (1 - b1) * g
        vel[:] = b2 * vel + (1 - b2) * g * g
        theta -= lr * mom / (np.sqrt(vel) + eps)
        return theta
    monkeypatch.setattr(SK, "adam_step", bad)
    assert _fails(skpins.test_adam_first_steps)


# ---- the counter-based Gaussian generator (oracle/philox.py)

def _philox_pins():
    import tests.test_philox_oracle as pp
    return pp


def test_philox_key_bumped_before_first_round_is_caught(monkeypatch):
    from oracle import philox as P
    pp = _philox_pins()
    orig = P.philox4x32_10
    monkeypatch.setattr(P, "philox4x32_10",
                        lambda ctr, key: orig(ctr, ((int(key[0]) + P.W0) & P.MASK32, (int(key[1]) + P.W1) & P.MASK32)))
    assert _fails(pp.test_philox_known_answer_vectors, 0)


def test_philox_swapped_multipliers_are_caught(monkeypatch):
    from oracle import philox as P
    pp = _philox_pins()
    monkeypatch.setattr(P, "M0", 0xCD9E8D57)
    monkeypatch.setattr(P, "M1", 0xD2511F53)
    assert _fails(pp.test_philox_known_answer_vectors, 2)


def test_box_muller_same_angle_function_is_caught(monkeypatch):
    from oracle import philox as P
    pp = _philox_pins()
    monkeypatch.setattr(P, "box_muller", lambda u1, u2: (np.sqrt(-2 * np.log(u1)) * np.cos(P.TWO_PI * u2),) * 2)
    assert _fails(pp.test_box_muller_closed_forms)
    assert _fails(pp.test_block_is_standard_normal)


def test_uniform_without_half_offset_is_caught(monkeypatch):
    from oracle import philox as P
    pp = _philox_pins()
    orig = P.uniform52
    monkeypatch.setattr(P, "uniform52", lambda a, b: orig(a, b) - 0.5 / 2.0 ** 52)
    assert _fails(pp.test_uniform52_closed_forms)


def test_single_pass_nystrom_mutations_are_caught(monkeypatch):
    """Single-pass Nystrom without the square of the singular values, or with the triangular
    solve on the wrong side (F C^T = Y), fails its pins."""
    import scipy.linalg as sla
    orig = O.nystrom_single_pass

    def no_square(applyA, G, k):
        U, t = orig(applyA, G, k)
        return U, np.sqrt(t)

    def wrong_side(applyA, G, k):
        G4 = O._orth(G)
        Y = applyA(G4)
        E = G4.T @ Y
        C = np.linalg.cholesky(0.5 * (E + E.T)).T
        F = sla.solve_triangular(C, Y.T, lower=False).T
        U, sig, _ = np.linalg.svd(F, full_matrices=False)
        return U[:, :k], sig[:k] ** 2

    for bad in (no_square, wrong_side):
        monkeypatch.setattr(O, "nystrom_single_pass", bad)
        assert _fails(pins.test_single_pass_nystrom_full_sketch_and_invariant_subspace)
        assert _fails(pins.test_single_pass_nystrom_closed_form_bounds_and_one_product)


def test_ritz_lmp_mutations_are_caught(monkeypatch):
    """The Ritz-LMP without its last term U Theta^{-1} U^T, or with Theta^{-1/2} for
    Theta^{-1}, and standard PCG with beta from r^T r instead of r^T z, fail their pins."""
    orig_dense, orig_apply, orig_pcg = O.ritz_lmp_dense, O.ritz_lmp_apply, O.pcg_standard

    def no_last_term(U, th, A):
        T = U @ np.diag(1.0 / th) @ U.T
        n = A.shape[0]
        return (np.eye(n) - T @ A) @ (np.eye(n) - A @ T)

    def half_power(U, th, A):
        return orig_dense(U, np.sqrt(th), A)

    for bad in (no_last_term, half_power):
        monkeypatch.setattr(O, "ritz_lmp_dense", bad)
        assert _fails(pins.test_ritz_lmp_identities)
    monkeypatch.setattr(O, "ritz_lmp_dense", orig_dense)

    def wrong_apply(U, th, AU, r):
        return orig_apply(U, th, AU, r) - U @ ((U.T @ r) / th)

    monkeypatch.setattr(O, "ritz_lmp_apply", wrong_apply)
    assert _fails(pins.test_ritz_lmp_identities)
    monkeypatch.setattr(O, "ritz_lmp_apply", orig_apply)

    def wrong_beta(applyA, b, precond, tol=1e-6, maxit=100):
        x = np.zeros_like(b)
        r = b.copy()
        z = precond(r)
        p = z.copy()
        rz = r @ z
        hJ = []
        for it in range(1, maxit + 1):
            Ap = applyA(p)
            alpha = rz / (p @ Ap)
            x = x + alpha * p
            r_new = r - alpha * Ap
            z = precond(r_new)
            beta = (r_new @ r_new) / (r @ r)
            r = r_new
            rz = r @ z
            p = z + beta * p
            hJ.append(-0.5 * (x @ (b + r)))
            if np.linalg.norm(r) <= tol * np.linalg.norm(b):
                break
        return O.PCGResult(x, it, True, np.linalg.norm(r) / np.linalg.norm(b), float("nan"), hJ[-1],
                           [], [], hJ, [], [])

    monkeypatch.setattr(O, "pcg_standard", wrong_beta)
    assert _fails(pins.test_standard_pcg_equals_split_pcg_and_cg)


def test_strong_constraint_mutations_are_caught(monkeypatch):
    """The strong-constraint adjoint sweep with M_i for M_i^T, or without B^{1/2} on its
    output, fails a pin."""
    orig = O.apply_A_sc

    def forward_in_adjoint(prob, X):
        X = np.asarray(X, dtype=np.float64)
        xs = [prob.Bsqrt @ X]
        for i in range(prob.N):
            xs.append(prob.M(i, xs[-1]))
        Zl = O._levels(prob, O.apply_HtRinvH(prob, np.concatenate(xs, axis=0)))
        w = Zl[prob.N]
        for i in range(prob.N - 1, -1, -1):
            w = Zl[i] + prob.M(i, w)
        return X + prob.Bsqrt @ w

    monkeypatch.setattr(O, "apply_A_sc", forward_in_adjoint)
    assert _fails(lambda: pins.test_strong_constraint_is_weak_constraint_without_model_error("advdiff"))
    assert _fails(pins.test_strong_constraint_dense_assembly_and_spectrum)

    def no_output_sqrt(prob, X):
        X = np.asarray(X, dtype=np.float64)
        return X + np.linalg.solve(prob.Bsqrt, orig(prob, X) - X)

    monkeypatch.setattr(O, "apply_A_sc", no_output_sqrt)
    assert _fails(lambda: pins.test_strong_constraint_is_weak_constraint_without_model_error("l96"))


def test_reorthogonalisation_mutations_are_caught(monkeypatch):
    """Reorthogonalisation against the last residual only, or a single projection with the
    earlier vectors unnormalised, each fail the ghost pin."""
    orig = O.pcg

    def last_only(applyA, b, x0=None, lmp=None, tol=1e-6, maxit=100, criterion=O.RES_TRUE,
                  keep_residuals=False, reorth=False):
        if not reorth:
            return orig(applyA, b, x0, lmp, tol, maxit, criterion, keep_residuals)
        x = np.zeros_like(b)
        r = b.copy()
        p = r.copy()
        rr = r @ r
        res, al, be = [r.copy()], [], []
        for _ in range(maxit):
            Ap = applyA(p)
            a = rr / (p @ Ap)
            x = x + a * p
            q = r / np.linalg.norm(r)
            r = r - a * Ap
            r = r - q * (q @ r)
            res.append(r.copy())
            rn = r @ r
            be.append(rn / rr)
            al.append(a)
            p = r + (rn / rr) * p
            rr = rn
        return O.PCGResult(x, maxit, False, 0.0, 0.0, 0.0, [], [], [], al, be, res)

    monkeypatch.setattr(O, "pcg", last_only)
    assert _fails(pins.test_cg_reorthogonalisation_removes_ghost_ritz_values)
    monkeypatch.setattr(O, "pcg", orig)

    def unnormalised(applyA, b, x0=None, lmp=None, tol=1e-6, maxit=100, criterion=O.RES_TRUE,
                     keep_residuals=False, reorth=False):
        if not reorth:
            return orig(applyA, b, x0, lmp, tol, maxit, criterion, keep_residuals)
        x = np.zeros_like(b)
        r = b.copy()
        p = r.copy()
        rr = r @ r
        res, al, be = [r.copy()], [], []
        for _ in range(maxit):
            Ap = applyA(p)
            a = rr / (p @ Ap)
            x = x + a * p
            r = r - a * Ap
            R = np.stack(res, axis=1)
            r = r - R @ (R.T @ r)
            res.append(r.copy())
            rn = r @ r
            be.append(rn / rr)
            al.append(a)
            p = r + (rn / rr) * p
            rr = rn
        return O.PCGResult(x, maxit, False, 0.0, 0.0, 0.0, [], [], [], al, be, res)

    monkeypatch.setattr(O, "pcg", unnormalised)
    assert _fails(pins.test_cg_reorthogonalisation_removes_ghost_ritz_values)


def test_lanczos_and_outer_loop_mutations_are_caught(monkeypatch):
    """Lanczos vectors without the alternating signs, T_j without the beta/alpha term on its
    diagonal, the outer loop's b with the wrong sign, and a trajectory that ignores the model
    error each fail a pin."""
    orig_tri, orig_pairs, orig_traj = O.cg_tridiagonal, O.cg_lanczos_pairs, O.forced_trajectory

    def no_signs(res, k, j=None):
        j = res.iters if j is None else j
        T = O.cg_tridiagonal(res.alphas, res.betas, j)
        F = np.stack([res.residuals[i] / np.linalg.norm(res.residuals[i]) for i in range(j)], axis=1)
        th, W = O._eig_desc(T)
        return F @ W[:, :k], th[:k]

    monkeypatch.setattr(O, "cg_lanczos_pairs", no_signs)
    assert _fails(pins.test_cg_tridiagonal_is_the_lanczos_projection)
    assert _fails(pins.test_cg_lanczos_pairs_converge_to_the_largest_eigenpairs)
    monkeypatch.setattr(O, "cg_lanczos_pairs", orig_pairs)

    def short_diag(alphas, betas, j):
        T = orig_tri(alphas, betas, j)
        return T - np.diag([0.0] + [betas[i - 1] / alphas[i - 1] for i in range(1, j)])

    monkeypatch.setattr(O, "cg_tridiagonal", short_diag)
    assert _fails(pins.test_cg_tridiagonal_is_the_lanczos_projection)
    monkeypatch.setattr(O, "cg_tridiagonal", orig_tri)

    orig_gn = O.gauss_newton

    def wrong_b_sign(prob, xb, y, n_outer, inner):
        orig_dinv = O.dinv_sqrt
        monkeypatch.setattr(O, "dinv_sqrt", lambda pr, v: -orig_dinv(pr, v))
        try:
            return orig_gn(prob, xb, y, n_outer, inner)
        finally:
            monkeypatch.setattr(O, "dinv_sqrt", orig_dinv)

    monkeypatch.setattr(O, "gauss_newton", wrong_b_sign)
    assert _fails(pins.test_gauss_newton_linear_model_converges_in_one_outer_loop)
    monkeypatch.setattr(O, "gauss_newton", orig_gn)

    monkeypatch.setattr(O, "forced_trajectory", lambda prob, x0, eta: orig_traj(prob, x0, 0.0 * eta))
    assert _fails(pins.test_gauss_newton_linear_model_converges_in_one_outer_loop)
