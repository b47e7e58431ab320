"""Planted mistakes: each is a plausible slip in the oracle (a dropped term, a
wrong sign or index, a transposed operand, a misread formula of the paper).
Each is written into a copy of the oracle's source, and the oracle's pin tests
(tests/test_oracle_*.py, which compare against closed forms, library routines,
brute force and the paper's theorems) are run against that copy in a fresh
interpreter; every mistake must make at least one pin fail.  The unmodified
copy must pass them all (the harness itself works)."""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lt_oracle.py")
PIN_FILES = sorted(os.path.join(ROOT, "tests", f) for f in os.listdir(os.path.join(ROOT, "tests"))
                   if f.startswith("test_oracle_") and f.endswith(".py") and f != "test_oracle_mutations.py")

# (name, exact text in the oracle, replacement)
MUTATIONS = [
    ("DCT delta_{i,j} as printed",
     "scale = np.sqrt((1.0 if i == 0 else 2.0) / n)", "scale = np.sqrt((1.0 if i == j else 2.0) / n)"),
    ("DCT matrix transposed",
     "C[i, j] = scale * np.cos(i * (2 * j + 1) * np.pi / (2.0 * n))",
     "C[j, i] = scale * np.cos(i * (2 * j + 1) * np.pi / (2.0 * n))"),
    ("DFT exponent sign", "np.exp(-2j * np.pi * i * j / n)", "np.exp(2j * np.pi * i * j / n)"),
    ("mode product contracts the wrong index",
     "np.tensordot(U, X, axes=([1], [ax]))", "np.tensordot(U, X, axes=([0], [ax]))"),
    ("inverse transform by the conjugate transpose",
     "Y = mode_product(Y, np.linalg.inv(M), i + 3)", "Y = mode_product(Y, M.conj().T, i + 3)"),
    ("slices numbered in row-major order",
     'flat = X.reshape((I1, I2, P), order="F")', 'flat = X.reshape((I1, I2, P), order="C")'),
    ("Hankel index off by one", "H[i, j] = 2 * n + 2 - s - 1", "H[i, j] = 2 * n + 1 - s - 1"),
    ("conjugate partner ignores the DFT", 'kk = (-k) % d if kind == "dft" else k', "kk = k"),
    ("SVT without the clamp", "s = np.maximum(s - tau, 0.0)", "s = np.abs(s - tau)"),
    ("DFT threshold scaled by alpha", "s = np.maximum(s - tau, 0.0)",
     "s = np.maximum(s - tau * (P if np.iscomplexobj(Ah) else 1), 0.0)"),
    ("DFT threshold scaled by sqrt(alpha)", "s = np.maximum(s - tau, 0.0)",
     "s = np.maximum(s - tau * (np.sqrt(P) if np.iscomplexobj(Ah) else 1), 0.0)"),
    ("truncation keeps one triplet too many", "kk = max(0, min(int(k), s.size))",
     "kk = max(0, min(int(k) + 1, s.size))"),
    ("nuclear norm without 1/alpha", "return singular_values(A, mats).sum() / transform_alpha(mats)",
     "return singular_values(A, mats).sum()"),
    ("alpha as the product of the alpha_i (not squared)", "alpha *= a2", "alpha *= np.sqrt(a2)"),
    ("gradient step sign as printed", "G = np.where(mask, M, Y)", "G = np.where(mask, -M, Y)"),
    ("gradient step drops the momentum point", "G = np.where(mask, M, Y)", "G = np.where(mask, M, X)"),
    ("momentum weight (t_k - 1)/t_k", "betas.append((t_prev - 1.0) / t)", "betas.append((t - 1.0) / t)"),
    ("momentum without the extrapolation", "Y = X + beta * (X - X_prev)", "Y = X + beta * (X_prev - X)"),
    ("threshold updated before its first use",
     "mus.append(fixed_mu if fixed_mu is not None else mu)\n        t_prev, t = t, (1.0 + np.sqrt(4.0 * t * t + 1.0)) / 2.0\n        mu = max(nu * mu, mu_bar)",
     "mu = max(nu * mu, mu_bar)\n        mus.append(fixed_mu if fixed_mu is not None else mu)\n        t_prev, t = t, (1.0 + np.sqrt(4.0 * t * t + 1.0)) / 2.0"),
    ("t_{k+1} recursion without the 4", "np.sqrt(4.0 * t * t + 1.0)", "np.sqrt(t * t + 1.0)"),
    ("stopping rule on ||X^{k+1} - X^k||", "crit = stop_criterion(Y, X_next)", "crit = stop_criterion(X, X_next)"),
    ("stopping rule normalised by ||Y||", "den = fro(X_next)", "den = fro(Y)"),
    ("stopping rule not gated", "if tol > 0 and crit <= tol and (at_floor or not gate_until_floor):",
     "if tol > 0 and crit <= tol:"),
    ("RSE squared as printed", "return fro(X_obt - X_ori) / fro(X_ori)",
     "return fro(X_obt - X_ori) ** 2 / fro(X_obt) ** 2"),
]

_RUNNER = r"""
import importlib.util, sys, types
path = sys.argv[1]
spec = importlib.util.spec_from_file_location("oracle.lt_oracle", path)
mod = importlib.util.module_from_spec(spec)
pkg = types.ModuleType("oracle")
pkg.__path__ = []
sys.modules["oracle"] = pkg
sys.modules["oracle.lt_oracle"] = mod
spec.loader.exec_module(mod)
for k, v in vars(mod).items():
    if not k.startswith("__"):
        setattr(pkg, k, v)
import pytest
sys.exit(pytest.main(["-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu", "--rootdir", sys.argv[2]]
                     + sys.argv[3:]))
"""


def _run_pins(source, tmp):
    path = os.path.join(tmp, "lt_oracle.py")
    with open(path, "w") as f:
        f.write(source)
    r = subprocess.run([sys.executable, "-c", _RUNNER, path, ROOT] + PIN_FILES, capture_output=True,
                       text=True, cwd=ROOT, timeout=600, env=dict(os.environ, PYTHONPATH=ROOT))
    return r.returncode, r.stdout[-2000:]


def test_every_planted_mistake_fails_a_pin():
    with open(SRC) as f:
        original = f.read()
    for name, old, new in MUTATIONS:
        assert original.count(old) >= 1, "mutation %r: text not found in the oracle" % name
    jobs = [("unmodified", original)] + [(name, original.replace(old, new, 1)) for name, old, new in MUTATIONS]
    with tempfile.TemporaryDirectory() as base:
        dirs = []
        for i in range(len(jobs)):
            d = os.path.join(base, str(i))
            os.makedirs(d)
            dirs.append(d)
        with ThreadPoolExecutor(max_workers=4) as ex:
            results = list(ex.map(lambda a: _run_pins(a[0][1], a[1]), zip(jobs, dirs)))
    rc0, out0 = results[0]
    assert rc0 == 0, "the unmodified oracle fails its pins:\n" + out0
    survivors = [name for (name, _), (rc, _) in zip(jobs[1:], results[1:]) if rc == 0]
    assert not survivors, "mistakes no pin catches: %s" % survivors
    # a collection or import error is not a caught mistake
    for (name, _), (rc, out) in zip(jobs[1:], results[1:]):
        assert rc == 1, "mutation %r: pytest exit %d (not a test failure)\n%s" % (name, rc, out)
