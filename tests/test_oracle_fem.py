"""The finite-element / adjoint oracle against its pins, and planted mistakes
in copies of it against the same pins (CPU only)."""
import importlib.util
import os
import sys

import pytest

from oracle import fem as F
from tests import pins_fem as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "fem.py")


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(pin):
    pin(F)


MUTANTS = {
    "volume_factor": ("np.abs(np.linalg.det(M)) / 6.0", "np.abs(np.linalg.det(M)) / 2.0"),
    "gradient_rows": ("grads = C[:, 1:, :]", "grads = C[:, :3, :]"),
    "gradient_transposed": ('np.einsum("eka,ekb->eab", grads, grads)', 'np.einsum("eak,ebk->eab", grads, grads)'),
    "assemble_ignores_nu": ("np.add.at(vals, pos, nu[m] * K[m, a, b])", "np.add.at(vals, pos, K[m, a, b])"),
    "assemble_upper_only": ("        for b in range(4):\n            m = (d[:, a]", "        for b in range(a, 4):\n            m = (d[:, a]"),
    "nu_grad_sign": ('return -np.einsum("ea,eab,eb->e", le, K, xe)', 'return np.einsum("ea,eab,eb->e", le, K, xe)'),
    "nu_grad_uses_x_twice": ("le, xe = _gather(np.asarray(lam, dtype=np.float64), d)",
                             "le, xe = _gather(np.asarray(x, dtype=np.float64), d)"),
    "csr_grad_transposed": ("        return -lam[line] * x[idx]\n", "        return -lam[idx] * x[line]\n"),
    "csc_grad_transposed": ("        return -lam[idx] * x[line]\n    g =", "        return -lam[line] * x[idx]\n    g ="),
    "sym_grad_drops_mirror": ("g = -(lam[line] * x[idx] + lam[idx] * x[line])", "g = -(lam[line] * x[idx])"),
    "sym_grad_diagonal_twice": ("    g[diag] = -lam[line[diag]] * x[idx[diag]]\n", ""),
    "adjoint_rhs_factor": ("lam = np.linalg.solve(A.T, 2.0 * r)", "lam = np.linalg.solve(A.T, r)"),
    "adjoint_rhs_sign": ("lam = np.linalg.solve(A.T, 2.0 * r)", "lam = np.linalg.solve(A.T, -2.0 * r)"),
    "cg_adjoint_rhs_factor": ("vals, 2.0 * r, tol=tol", "vals, r, tol=tol"),
    "gather_ignores_mask": ("    out[m] = v[d[m]]\n", "    out[m] = v[d[m]]\n    out[~m] = v[0]\n"),
}


def _load_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    path = tmp_path / f"fem_{name}.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"fem_mutant_{name}", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_caught(name, tmp_path):
    mod = _load_mutant(name, tmp_path)
    failed = P.run_all(mod)
    assert failed, f"planted mistake {name} passes every pin"
