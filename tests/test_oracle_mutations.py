"""Mutation check of the oracle's pins (CPU).

Each case plants one plausible mistake in a copy of an oracle module's source
(a dropped term, a wrong sign, scale or index, a missing update), loads the
mutant in place of the real module and runs the pins of test_oracle_pins.py
against it.  At least one pin must fail for every mutant: a mistake anywhere in
the oracle's arithmetic has to be caught by something other than the oracle.
The real modules and the pins themselves are not modified.
"""

import importlib.util
import os
import types

import numpy as np
import pytest

import oracle
from oracle import bcd as real_bcd, exact as real_exact, sampler as real_sampler

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_DIR = os.path.dirname(os.path.abspath(oracle.__file__))


def _pins():
    spec = importlib.util.spec_from_file_location("_oracle_pins_for_mutation",
                                                  os.path.join(HERE, "test_oracle_pins.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


PINS = _pins()


def _mutant(modname, old, new):
    path = os.path.join(ORACLE_DIR, modname + ".py")
    src = open(path).read()
    assert src.count(old) == 1, f"mutation site not unique in {modname}.py: {old!r}"
    src = src.replace(old, new, 1)
    m = types.ModuleType(f"oracle._mutant_{modname}")
    m.__package__ = "oracle"
    m.__file__ = path
    exec(compile(src, path + " (mutant)", "exec"), m.__dict__)
    return m


def _dual_small():
    import synth
    X, y, _ = synth.gaussian_ridge(30, 200, 21)
    return X.numpy(), y.numpy(), 0.05


# The pins run against each mutant, cheapest first.
def _pin_calls():
    ds = _dual_small()
    return [
        ("gram integer exact", PINS.test_gram_integer_exact_and_orientation, ()),
        ("exact primal s=1", PINS.test_fp64_oracle_matches_exact_primal, (1,)),
        ("exact primal s=3", PINS.test_fp64_oracle_matches_exact_primal, (3,)),
        ("exact dual s=1", PINS.test_fp64_oracle_matches_exact_dual, (1,)),
        ("exact dual s=5", PINS.test_fp64_oracle_matches_exact_dual, (5,)),
        ("exact CA-BCD = BCD s=3", PINS.test_exact_cabcd_equals_bcd, (3,)),
        ("exact CA-BDCD = BDCD s=3", PINS.test_exact_cabdcd_equals_bdcd, (3,)),
        ("block minimiser", PINS.test_block_step_is_block_minimiser, ()),
        ("dual block minimiser", PINS.test_dual_block_step_is_block_minimiser, ()),
        ("full block newton", PINS.test_full_block_is_one_newton_step, ()),
        ("orthogonal design", PINS.test_orthogonal_design_decouples, ()),
        ("duality identity", PINS.test_duality_identity_and_dual_optimum, (ds,)),
        ("splitmix64 golden", PINS.test_splitmix64_reference_outputs, ()),
        ("lemire power of two", PINS.test_lemire_power_of_two_is_top_bits, ()),
        ("lemire rejection", PINS.test_lemire_rejection_removes_bias, ()),
        ("blocks distinct", PINS.test_blocks_distinct_and_in_range, (64, 4)),
        ("subsets uniform", PINS.test_subsets_uniform_chi2, ()),
    ]


MUTATIONS = [
    # (name, module, source text, replacement)
    ("primal: dropped lambda S_jt term", "bcd",
     "rhs -= lam * (_overlap(blocks[j], blocks[t]) @ deltas[t])", "pass"),
    ("primal: dropped cross Gram term", "bcd",
     "rhs -= G[J, T] @ deltas[t]", "pass"),
    ("primal: transposed cross block", "bcd",
     "rhs -= G[J, T] @ deltas[t]", "rhs -= G[J, T].T @ deltas[t]"),
    ("primal: sign of X y", "bcd",
     "+ Xy[blocks[j]] / n", "- Xy[blocks[j]] / n"),
    ("primal: lambda w term dropped", "bcd",
     "rhs = -lam * w[blocks[j]] - Yz[J] / n", "rhs = - Yz[J] / n"),
    ("primal: Gram scaled by 1/n twice", "bcd",
     "G = (Y @ Y.T) / n + lam * np.eye(sk * b)", "G = (Y @ Y.T) / (n * n) + lam * np.eye(sk * b)"),
    ("primal: 2 lambda on the Gram diagonal", "bcd",
     "G = (Y @ Y.T) / n + lam * np.eye(sk * b)", "G = (Y @ Y.T) / n + 2 * lam * np.eye(sk * b)"),
    ("primal: missing z update", "bcd", "z = z + X.T @ v", "z = z"),
    ("primal: overwrite instead of scatter-add", "bcd",
     "                v[i] += deltas[t][u]\n        w = w + v",
     "                v[i] = deltas[t][u]\n        w = w + v"),
    ("dual: cross term scale 1/(lam n^2)", "bcd",
     "rhs += (YtY[J, T] @ deltas[t]) / (lam * n)",
     "rhs += (YtY[J, T] @ deltas[t]) / (lam * n * n)"),
    ("dual: overlap sign", "bcd",
     "rhs += _overlap(blocks[j], blocks[t]) @ deltas[t]",
     "rhs -= _overlap(blocks[j], blocks[t]) @ deltas[t]"),
    ("dual: sign of y", "bcd",
     "rhs = -Ytw[J] + alpha[blocks[j]] + y[blocks[j]]",
     "rhs = -Ytw[J] + alpha[blocks[j]] - y[blocks[j]]"),
    ("dual: update sign of w", "bcd",
     "w = w - np.asarray(X @ v).ravel() / (lam * n)",
     "w = w + np.asarray(X @ v).ravel() / (lam * n)"),
    ("dual: Theta shift lambda instead of 1/n", "bcd",
     "Gp = YtY / (lam * n * n) + np.eye(sk * b) / n",
     "Gp = YtY / (lam * n * n) + lam * np.eye(sk * b)"),
    ("dual: delta missing the -1/n", "bcd",
     "deltas.append(-_chol_solve(Theta, rhs) / n)", "deltas.append(_chol_solve(Theta, rhs) / n)"),
    ("objective: lambda/2 written lambda", "bcd",
     "return 0.5 * float(r @ r) / n + 0.5 * lam * float(w @ w)",
     "return 0.5 * float(r @ r) / n + lam * float(w @ w)"),
    ("dual objective: 1/n on ||a + y||^2 dropped", "bcd",
     "return 0.5 * lam * float(v @ v) + 0.5 * float(a @ a) / n",
     "return 0.5 * lam * float(v @ v) + 0.5 * float(a @ a)"),
    ("closed form: 2 lambda", "bcd",
     "M = XXt / n + lam * np.eye(d)", "M = XXt / n + 2 * lam * np.eye(d)"),
    ("gram: shift on every entry", "bcd",
     "G = scale * (Y @ Y.T) + shift * np.eye(len(idx))",
     "G = scale * (Y @ Y.T) + shift * np.ones((len(idx), len(idx)))"),
    ("gram: rows of the transpose", "bcd",
     "Yu = None if u is None else Y @ np.asarray(u, dtype=np.float64)",
     "Yu = None if u is None else (Y @ np.asarray(u, dtype=np.float64))[::-1]"),
    ("sampler: mix64 second constant", "sampler",
     "* 0x94D049BB133111EB)", "* 0x94D049BB133111EA)"),
    ("sampler: no Lemire rejection", "sampler",
     "while low < threshold:", "while False:"),
    ("sampler: Floyd keeps duplicates", "sampler",
     "out.append(j if v in out else v)", "out.append(v)"),
    ("exact: CA overlap term dropped", "exact",
     "val -= lam * deltas[t][v]", "pass"),
    ("exact: dual BDCD step sign", "exact",
     "da = [-v / n for v in _solve(Th, rhs)]", "da = [v / n for v in _solve(Th, rhs)]"),
]


@pytest.mark.parametrize("name,modname,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_fails_a_pin(monkeypatch, name, modname, old, new):
    mutant = _mutant(modname, old, new)
    real = {"bcd": real_bcd, "exact": real_exact, "sampler": real_sampler}
    # the pins see the mutant; the FP64 oracle also draws its blocks through
    # the sampler it imported, so a sampler mutant replaces that name too
    monkeypatch.setattr(PINS, modname, mutant)
    if modname == "sampler":
        monkeypatch.setattr(real_bcd, "sample_block", mutant.sample_block)
    failed = []
    for pin_name, fn, args in _pin_calls():
        try:
            with np.errstate(all="ignore"):
                fn(*args)
        except Exception:   # an assertion, or an error the mutant raises
            failed.append(pin_name)
            break
    assert failed, f"no pin caught the mutation '{name}'"
    assert real[modname] is not mutant
