"""Plants plausible mistakes in the oracle (CPU only) and checks that the pins catch
each one, so that the pins are known to constrain the parts they claim to."""
import numpy as np
import pytest

import oracle as O
import oracle.dpd_pa as OC
import test_oracle_grad as TG
import test_oracle_pins as TP


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def _all_pins():
    return [TP.test_gmp_linear_gain_only, TP.test_gmp_fir_matches_numpy_convolve,
            TP.test_gmp_memoryless_constant_envelope_closed_form, TP.test_gmp_lag_term_direction,
            TP.test_gmp_lead_term_direction, TP.test_gmp_brute_force_tiny,
            TP.test_gmp_least_squares_identification, TP.test_linear_pa_identity_dpd_zero_error,
            TP.test_features_exact_values_and_taps, TP.test_tdnn_hand_evaluated_single_neuron,
            TP.test_tdnn_weight_orientation, TP.test_stream_start_equals_zero_prefix,
            lambda: TG.test_gradient_matches_torch_autograd_fp64(
                dict(T=3, nl=2, H=5, K=5, M=3, L=2, N=64))]


def _caught(monkeypatch, target, name, replacement):
    monkeypatch.setattr(target, name, replacement)
    caught = [p for p in _all_pins() if _fails(p)]
    monkeypatch.undo()
    return caught


def test_swapped_lag_and_lead_is_caught(monkeypatch):
    orig = OC.gmp_terms

    def swapped(K, M, L):
        return [(f, k, l, g, (l - g if f == "b" else l + g if f == "c" else d))
                for f, k, l, g, d in orig(K, M, L)]
    assert _caught(monkeypatch, OC, "gmp_terms", swapped)


def test_dropped_lead_family_is_caught(monkeypatch):
    orig = OC.gmp_terms
    assert _caught(monkeypatch, OC, "gmp_terms",
                   lambda K, M, L: [t for t in orig(K, M, L) if t[0] != "c"])


def test_off_by_one_delay_is_caught(monkeypatch):
    orig = OC.delay
    assert _caught(monkeypatch, OC, "delay", lambda v, d: orig(v, d + 1 if d > 0 else d))


def test_wrong_feature_power_is_caught(monkeypatch):
    def bad_features(x, taps):
        cols = []
        for t in range(taps):
            z = OC.delay(x, t)
            m = np.abs(z)
            cols += [z.real, z.imag, m, m * m, m * m]        # |z|^2 instead of |z|^3
        return np.stack(cols, axis=1)
    assert _caught(monkeypatch, OC, "features", bad_features)


def test_transposed_weights_is_caught(monkeypatch):
    orig = OC.unpack_tdnn

    def transposed(w, taps, n_hidden, hidden):
        layers = orig(w, taps, n_hidden, hidden)
        out = []
        for W, b in layers:
            fo, fi = W.shape
            out.append((W.reshape(-1).reshape(fi, fo).T.copy(), b))
        return out
    assert _caught(monkeypatch, OC, "unpack_tdnn", transposed)


def test_missing_tanh_derivative_is_caught(monkeypatch):
    def bad_backward(hs, layers, g_u):
        delta = np.stack([g_u.real, g_u.imag], axis=1)
        grads = [None] * len(layers)
        for i in range(len(layers) - 1, -1, -1):
            W, _ = layers[i]
            grads[i] = (delta.T @ hs[i], delta.sum(axis=0))
            if i > 0:
                delta = delta @ W                              # forgot (1 - h^2)
        return grads
    assert _caught(monkeypatch, OC, "tdnn_backward", bad_backward)


def test_gmp_backward_missing_envelope_term_is_caught(monkeypatch):
    def bad(u, g_y, a, b, c):
        K, M1 = a.shape
        L = b.shape[2] if b.size else 0
        r = np.abs(u)
        g_u = np.zeros_like(u)
        for fam, k, l, g, d in OC.gmp_terms(K, M1 - 1, L):
            cf = OC._coef(a, b, c, fam, k, l, g)
            g_u += OC.advance(np.conj(cf) * OC.delay(r, d) ** k * g_y, l)
        return g_u
    assert _caught(monkeypatch, OC, "gmp_backward", bad)


# ---------------------------------------------------------------- ACPR plan, ridge
import oracle.spectrum as OS
import test_oracle_ila as TI


def _acpr_pins():
    return ([lambda k=k, b=b: TP.test_band_plan_single_bin_membership(k, b)
             for k, b in [(0, "M"), (20, "M"), (-20, "M"), (21, "U"), (60, "U"), (-21, "L"),
                          (-60, "L"), (61, None), (-61, None)]]
            + [TP.test_band_plan_exact_sums_of_distinct_bins, TP.test_acpr_of_tones_in_known_channels])


def _plan(main_hi, up_lo, up_hi, lo_lo, lo_hi, swap=False):
    """A band_powers variant: main |k| <= main_hi, upper up_lo <= k <= up_hi, lower
    lo_lo <= k <= lo_hi (bins as signed indices), optionally with L and U swapped."""
    def bp(psd, h):
        nfft = psd.size
        k = np.arange(nfft)
        ks = np.where(k < nfft // 2, k, k - nfft)
        main = psd[np.abs(ks) <= main_hi(h)].sum()
        up = psd[(ks >= up_lo(h)) & (ks <= up_hi(h))].sum()
        lo = psd[(ks >= lo_lo(h)) & (ks <= lo_hi(h))].sum()
        return (float(up), float(main), float(lo)) if swap else (float(lo), float(main), float(up))
    return bp


@pytest.mark.parametrize("name,variant", [
    ("adjacent width h", _plan(lambda h: h, lambda h: h + 1, lambda h: 2 * h, lambda h: -2 * h, lambda h: -h - 1)),
    ("L and U swapped", _plan(lambda h: h, lambda h: h + 1, lambda h: 3 * h, lambda h: -3 * h, lambda h: -h - 1, swap=True)),
    ("main edge |k| < h", _plan(lambda h: h - 1, lambda h: h, lambda h: 3 * h, lambda h: -3 * h, lambda h: -h)),
    ("main edge |k| <= h + 1", _plan(lambda h: h + 1, lambda h: h + 2, lambda h: 3 * h, lambda h: -3 * h, lambda h: -h - 2)),
    ("outer edge 3h excluded", _plan(lambda h: h, lambda h: h + 1, lambda h: 3 * h - 1, lambda h: -3 * h + 1, lambda h: -h - 1)),
    ("outer edge 3h + 1 included", _plan(lambda h: h, lambda h: h + 1, lambda h: 3 * h + 1, lambda h: -3 * h - 1, lambda h: -h - 1)),
])
def test_acpr_plan_mistakes_are_caught(monkeypatch, name, variant):
    monkeypatch.setattr(OS, "band_powers", variant)
    caught = [p for p in _acpr_pins() if _fails(p)]
    monkeypatch.undo()
    assert caught, name


def test_acpr_plan_pins_pass_unmutated():
    assert not [p for p in _acpr_pins() if _fails(p)]


@pytest.mark.parametrize("name", ["no /J", "Frobenius of G", "ridge on the right-hand side"])
def test_ridge_mistakes_are_caught(monkeypatch, name):
    import oracle.ila as I

    def bad(G, b, ridge=0.0):
        J = G.shape[0]
        A = G.copy()
        rhs = b.copy()
        if ridge:
            if name == "no /J":
                A += ridge * np.trace(G).real * np.eye(J)
            elif name == "Frobenius of G":
                A += ridge * np.linalg.norm(G) / J * np.eye(J)
            else:
                A += ridge * np.trace(G).real / J * np.eye(J)
                rhs = rhs * (1 + ridge)
        return np.linalg.solve(A, rhs)
    monkeypatch.setattr(I, "solve_normal", bad)
    pins = [lambda r=r: TI.test_ridge_equals_least_squares_on_augmented_system(r) for r in (1e-3, 0.3)]
    caught = [p for p in pins if _fails(p)]
    monkeypatch.undo()
    assert caught, name
