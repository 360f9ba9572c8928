"""The oracle's pins catch plausible mistakes.  Each case plants one mistake
in a copy of an oracle module (a dropped factor or term, a wrong sign, a
wrong or transposed index, a missing weight, another orthonormalisation),
substitutes the copy for the module the pins in test_oracle.py use, and
requires that at least one of the named pins fails on it.  The mistakes are
planted in the oracle only, on the CPU."""
import os
import types

import numpy as np
import pytest

import oracle
from paper_2304_07006_amd import inputs

import test_oracle as pins

ORACLE_DIR = os.path.dirname(os.path.abspath(oracle.__file__))


@pytest.fixture(scope="module")
def tierA(tiny):
    from oracle import explicit as ex
    return ex.tier_a(tiny.xyz, tiny.w, tiny.phi, tiny.occ, tiny.jastrow)


def mutant(name, old, new, nth=0):
    """oracle.<name> with the nth occurrence of `old` replaced by `new`."""
    path = os.path.join(ORACLE_DIR, name + ".py")
    src = open(path).read()
    at = -1
    for _ in range(nth + 1):
        at = src.index(old, at + 1)
    src = src[:at] + new + src[at + len(old):]
    mod = types.ModuleType(f"oracle.{name}")
    mod.__package__ = "oracle"
    mod.__file__ = path
    exec(compile(src, path, "exec"), mod.__dict__)
    return mod


def caught(checks):
    """True when at least one of the pin calls raises AssertionError."""
    for check in checks:
        try:
            check()
        except AssertionError:
            return True
    return False


# ---------------------------------------------------------------- tier B --
FACTORISED = [
    # (why, old, new, occurrence)
    ("W without the spin factor two", 'W = 2.0 * np.einsum("xitu,tu->xi", K, gamma)',
     'W = 1.0 * np.einsum("xitu,tu->xi", K, gamma)', 0),
    ("A = V~ + Z~ (sign)", "A = Vt - Zt", "A = Vt + Zt", 0),
    ("B without the 1/2", "B = 0.5 * Wt[None, :, None, None] * K - Z", "B = Wt[None, :, None, None] * K - Z", 0),
    ("Y with its indices swapped", 'Y = np.einsum("xiru,tu->xirt", K, gamma)',
     'Y = np.einsum("xiru,tu->xitr", K, gamma)', 0),
    ("Z without its Y rho term", '+ np.einsum("xirt,its->xirs", Y, rho))', '+ 0.0 * np.einsum("xirt,its->xirs", Y, rho))', 0),
    ("no (pq)<->(rs) permutation", "V2 = -(f + f.T).reshape(N, N, N, N)", "V2 = -(2.0 * f).reshape(N, N, N, N)", 0),
    ("exchange term of Delta h with the direct index", '- np.einsum("psrq,rs->pq", V2, gamma))',
     '- np.einsum("pqrs,rs->pq", V2, gamma))', 0),
    ("zero-body factor 1/3 for 2/3", "return -(2.0 / 3.0) * float(", "return -(1.0 / 3.0) * float(", 0),
    ("pair density without the grid weight", "rho = w[rows, None, None] * phi[:, rows].T[:, :, None]",
     "rho = phi[:, rows].T[:, :, None]", 0),
    ("K without the weight of g'", "rho_j = ((phi * w)[:, None, :] * phi[None, :, :])",
     "rho_j = ((phi)[:, None, :] * phi[None, :, :])", 1),
]


@pytest.mark.parametrize("why,old,new,nth", FACTORISED, ids=[c[0] for c in FACTORISED])
def test_tier_b_mistake_is_caught(monkeypatch, tiny, tierA, why, old, new, nth):
    monkeypatch.setattr(pins, "fb", mutant("factorised", old, new, nth))
    assert caught([lambda: pins.test_tier_a_equals_tier_b(tiny, tierA)]), why


# --------------------------------------------------------------- Jastrow --
JASTROW = [
    ("Pade u' with the power 3", "return 1.0 / (2.0 * (1.0 + b * r) ** 2)", "return 1.0 / (2.0 * (1.0 + b * r) ** 3)", 0),
    ("power-series u' without the factor k+1", "s = sum((k + 1) * c * t ** k for k, c in enumerate(coef))",
     "s = sum(c * t ** k for k, c in enumerate(coef))", 0),
    ("grad_2 for grad_1 (difference reversed)",
     "np.subtract(np.ascontiguousarray(xa.T)[:, :, None], np.ascontiguousarray(xb.T)[:, None, :], out=d)",
     "np.subtract(np.ascontiguousarray(xb.T)[:, None, :], np.ascontiguousarray(xa.T)[:, :, None], out=d)", 0),
    ("Pade u with (1 + b r) squared", "return r / (2.0 * (1.0 + b * r))", "return r / (2.0 * (1.0 + b * r) ** 2)", 0),
]


@pytest.mark.parametrize("why,old,new,nth", JASTROW, ids=[c[0] for c in JASTROW])
def test_jastrow_mistake_is_caught(monkeypatch, why, old, new, nth):
    monkeypatch.setattr(pins, "oj", mutant("jastrow", old, new, nth))
    checks = [lambda j=j: pins.test_du_matches_finite_difference(j)
              for j in (pins.J("pade", 1.0, ()), pins.J("pade", 0.3, ()),
                        pins.J("power", 0.0, (0.5, -0.1, 0.07, 0.02)))]
    checks += [pins.test_pade_b1_equals_power_half, pins.test_grad1_antisymmetric_zero_on_diagonal_and_bounded,
               pins.test_grad1_matches_finite_difference_of_u]
    assert caught(checks), why


# ---------------------------------------------------------------- Loewdin --
LOWDIN = [
    ("S^-1 for S^-1/2", "C = (U / np.sqrt(lam)) @ U.T", "C = (U / lam) @ U.T", 0),
    ("overlap without the grid weights", "return (chi * w) @ chi.T", "return chi @ chi.T", 0),
    ("Gram-Schmidt (Cholesky) for Loewdin", "C = (U / np.sqrt(lam)) @ U.T",
     "C = np.linalg.inv(np.linalg.cholesky(S))", 0),
    ("eigenvectors transposed", "C = (U / np.sqrt(lam)) @ U.T", "C = (U.T / np.sqrt(lam)) @ U", 0),
]


@pytest.mark.parametrize("why,old,new,nth", LOWDIN, ids=[c[0] for c in LOWDIN])
def test_lowdin_mistake_is_caught(monkeypatch, why, old, new, nth):
    ol = mutant("lowdin", old, new, nth)
    monkeypatch.setattr(pins, "ol", ol)
    p = inputs.make_problem(24, 3, 4000, 3, "chain", "pade", seed=31)
    phi, C, lam = ol.lowdin(p.chi, p.w)
    case = (p, phi, C, lam, (p.chi * p.w) @ p.chi.T)
    checks = [lambda: pins.test_lowdin_matrix_is_symmetric_positive_definite_inverse_square_root(case),
              lambda: pins.test_lowdin_orbitals_orthonormal_under_weights(case),
              lambda: pins.test_lowdin_is_the_closest_orthonormal_set(case),
              pins.test_lowdin_two_function_closed_form]
    assert caught(checks), why


# ----------------------------------------------------------- the gradient --
GRADIENT = [
    ("central difference without the 1/2", "g[k] = 0.5 * (loss(xyz, w, phi, occ, coef + e, D, G)",
     "g[k] = 1.0 * (loss(xyz, w, phi, occ, coef + e, D, G)", 0),
    ("loss without the one-body weight", "return E0 + float(np.sum(h1 * D)) + float(np.sum(V2 * G))",
     "return E0 + float(np.sum(V2 * G))", 0),
]


@pytest.mark.parametrize("why,old,new,nth", GRADIENT, ids=[c[0] for c in GRADIENT])
def test_gradient_mistake_is_caught(monkeypatch, why, old, new, nth):
    og = mutant("gradient", old, new, nth)
    monkeypatch.setattr(pins, "og", og)
    assert caught([pins.test_loss_homogeneous_quadratic_and_gradient,
                   pins.test_loss_weights_select_the_outputs]), why


# the same pin groups pass on unmodified copies (so a caught mistake is the mistake's doing)
def test_unmodified_copies_pass_every_pin_group(monkeypatch, tiny, tierA):
    monkeypatch.setattr(pins, "fb", mutant("factorised", "import numpy as np", "import numpy as np"))
    assert not caught([lambda: pins.test_tier_a_equals_tier_b(tiny, tierA)])
    monkeypatch.setattr(pins, "oj", mutant("jastrow", "import numpy as np", "import numpy as np"))
    checks = [lambda j=j: pins.test_du_matches_finite_difference(j)
              for j in (pins.J("pade", 1.0, ()), pins.J("pade", 0.3, ()),
                        pins.J("power", 0.0, (0.5, -0.1, 0.07, 0.02)))]
    checks += [pins.test_pade_b1_equals_power_half, pins.test_grad1_antisymmetric_zero_on_diagonal_and_bounded,
               pins.test_grad1_matches_finite_difference_of_u]
    assert not caught(checks)
    ol = mutant("lowdin", "import numpy as np", "import numpy as np")
    monkeypatch.setattr(pins, "ol", ol)
    p = inputs.make_problem(24, 3, 4000, 3, "chain", "pade", seed=31)
    phi, C, lam = ol.lowdin(p.chi, p.w)
    case = (p, phi, C, lam, (p.chi * p.w) @ p.chi.T)
    assert not caught([lambda: pins.test_lowdin_matrix_is_symmetric_positive_definite_inverse_square_root(case),
                       lambda: pins.test_lowdin_orbitals_orthonormal_under_weights(case),
                       lambda: pins.test_lowdin_is_the_closest_orthonormal_set(case),
                       pins.test_lowdin_two_function_closed_form])
    monkeypatch.setattr(pins, "og", mutant("gradient", "import numpy as np", "import numpy as np"))
    assert not caught([pins.test_loss_homogeneous_quadratic_and_gradient, pins.test_loss_weights_select_the_outputs])


# --------------------------------------------------- tier A (explicit L) --
EXPLICIT = [
    ("L without its electron-2-centred term", "L = L1 + L2 + L3", "L = L1 + L3", 0),
    ("eq. dU with a wrong sign", '- np.einsum("prtqus,tu->prqs", L, g, optimize=True)',
     '+ np.einsum("prtqus,tu->prqs", L, g, optimize=True)', 0),
    ("eq. dU with an exchanged index", 'np.einsum("prtusq,tu->prqs", L, g, optimize=True))',
     'np.einsum("prtuqs,tu->prqs", L, g, optimize=True))', 0),
    ("grid intermediate without the weight", "pw = phi * w                                   # [N][j]",
     "pw = phi                                       # [N][j]", 0),
]


@pytest.mark.parametrize("why,old,new,nth", EXPLICIT, ids=[c[0] for c in EXPLICIT])
def test_tier_a_mistake_is_caught(monkeypatch, tiny, why, old, new, nth):
    ex = mutant("explicit", old, new, nth)
    monkeypatch.setattr(pins, "ex", ex)
    A = ex.tier_a(tiny.xyz, tiny.w, tiny.phi, tiny.occ, tiny.jastrow)
    checks = [lambda: pins.test_tier_a_equals_tier_b(tiny, A),
              lambda: pins.test_determinant_brute_force(tiny, A),
              lambda: pins.test_K_two_point_closed_form()]
    assert caught(checks), why


# ------------------------------------------------------ the TC integrals --
TC2 = [
    ("without the electron-swap term of B", "return (A + B + B.T).reshape(N, N, N, N)",
     "return (A + 2.0 * B).reshape(N, N, N, N)", 0),
    ("gradient term without its factor 2", 't2 = 2.0 * np.einsum("pg,xqg,xgh,rh,sh->pqrs"',
     't2 = 1.0 * np.einsum("pg,xqg,xgh,rh,sh->pqrs"', 0),
    ("definition without its 1/2", "return 0.5 * (t1 + t2 + t3 + t4)", "return (t1 + t2 + t3 + t4)", 0),
    ("quadratic part without the weights", "rho = ((phi * w)[:, None, :] * phi[None, :, :]).reshape(phi.shape[0] ** 2, -1)",
     "rho = ((phi)[:, None, :] * phi[None, :, :]).reshape(phi.shape[0] ** 2, -1)", 0),
]


@pytest.mark.parametrize("why,old,new,nth", TC2, ids=[c[0] for c in TC2])
def test_tc_integral_mistake_is_caught(monkeypatch, why, old, new, nth):
    import sys
    tc2 = mutant("tc2", old, new, nth)
    monkeypatch.setitem(sys.modules, "oracle.tc2", tc2)
    monkeypatch.setattr(oracle, "tc2", tc2, raising=False)
    p = inputs.make_problem(8, 2, 80, 2, "pair", "power16", seed=13)
    case = (p, inputs.orbital_gradients(p))
    checks = [lambda: pins.test_tc_two_body_factorised_equals_definition(case),
              lambda: pins.test_tc_two_body_linear_and_quadratic_parts(case)]
    assert caught(checks), why


def test_unmodified_tier_a_and_tc_copies_pass_their_pins(monkeypatch, tiny):
    import sys
    ex = mutant("explicit", "import numpy as np", "import numpy as np")
    monkeypatch.setattr(pins, "ex", ex)
    A = ex.tier_a(tiny.xyz, tiny.w, tiny.phi, tiny.occ, tiny.jastrow)
    assert not caught([lambda: pins.test_tier_a_equals_tier_b(tiny, A),
                       lambda: pins.test_determinant_brute_force(tiny, A),
                       lambda: pins.test_K_two_point_closed_form()])
    tc2 = mutant("tc2", "import numpy as np", "import numpy as np")
    monkeypatch.setitem(sys.modules, "oracle.tc2", tc2)
    monkeypatch.setattr(oracle, "tc2", tc2, raising=False)
    p = inputs.make_problem(8, 2, 80, 2, "pair", "power16", seed=13)
    case = (p, inputs.orbital_gradients(p))
    assert not caught([lambda: pins.test_tc_two_body_factorised_equals_definition(case),
                       lambda: pins.test_tc_two_body_linear_and_quadratic_parts(case)])
