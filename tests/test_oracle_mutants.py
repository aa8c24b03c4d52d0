"""Planted mistakes in the oracle must trip at least one pin.

Each case edits one spot of oracle.c (a dropped term, a wrong sign, index or
coefficient), builds that copy in a temporary directory, and runs every pin
against it in a child process.  A mutant that passes all pins would mean the
pins cannot tell that mistake from the right answer.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "force_sign_x": ("const double dx = x[j] - xi,", "const double dx = xi - x[j],"),
    "force_r2_power": ("const double mr3 = m[j] * rinv * rinv2;", "const double mr3 = m[j] * rinv2;"),
    "force_index_vy": ("dvy = v[n + j] - vyi", "dvy = v[j] - vyi"),
    "softening_not_squared": ("const double eps2 = eps * eps;\n#pragma omp parallel for schedule(dynamic, 16)\n    for (int64_t q = 0; q < n_act; ++q) {\n        double a[3], k[3], p;",
                              "const double eps2 = eps;\n#pragma omp parallel for schedule(dynamic, 16)\n    for (int64_t q = 0; q < n_act; ++q) {\n        double a[3], k[3], p;"),
    "jerk_drop_radial": ("kx += mr3 * (dvx - c * dx);", "kx += mr3 * dvx;"),
    "jerk_coeff": ("const double c = 3.0 * rv * rinv2;", "const double c = 2.0 * rv * rinv2;"),
    "pot_self_term": ("        if (j == i) continue;\n        const double dx", "        const double dx"),
    "pot_sign": ("ph -= m[j] * rinv;", "ph += m[j] * rinv;"),
    "predict_drop_jerk": ("+ k[o] * h * h * h / 6.0;", ";"),
    "predict_vel_coeff": ("vp[o] = v[o] + a[o] * h + k[o] * h * h / 2.0;", "vp[o] = v[o] + a[o] * h + k[o] * h * h / 6.0;"),
    "correct_swap_k": ("(4.0 * k0[d] + 2.0 * k1[d])", "(2.0 * k0[d] + 4.0 * k1[d])"),
    "correct_da_sign": ("const double da = a0[d] - a1[d];", "const double da = a1[d] - a0[d];"),
    "correct_x_coeff": ("a3[d] * h5 / 120.0;", "a3[d] * h5 / 60.0;"),
    "aarseth_no_propagation": ("a2p[d] = a2[d] + a3[d] * h;", "a2p[d] = a2[d];"),
    "aarseth_k_squared": ("(na * na2 + nk * nk)", "(na * na2 + nk)"),
    "quantize_no_commensurability": ("dt_new >= 2.0 * dt_old && fmod(t_now, 2.0 * dt_old) == 0.0", "dt_new >= 2.0 * dt_old"),
    "quantize_free_growth": ("        dt_new = 2.0 * dt_old;\n    } else {", "        ;\n    } else {"),
    "slice_drop_last": ("if (e > n) e = n;", "if (e > n) e = n - 1;"),
    "abs_drop_mass_factor": ("sa += mr3 * sqrt(dx * dx + dy * dy + dz * dz);", "sa += sqrt(dx * dx + dy * dy + dz * dz);"),
    "abs_drop_radial_jerk": ("const double wx = dvx - c * dx,", "const double wx = dvx,"),
    "abs_jerk_coeff": ("const double c = 3.0 * (dx * dvx + dy * dvy + dz * dvz) * rinv * rinv;",
                       "const double c = 2.0 * (dx * dvx + dy * dvy + dz * dvz) * rinv * rinv;"),
    "abs_pot_power": ("sp += m[j] * rinv;", "sp += m[j] * rinv * rinv;"),
    "abs_self_term": ("        double sa = 0.0, sk = 0.0, sp = 0.0;\n        for (int64_t j = 0; j < n; ++j) {\n            if (j == i) continue;",
                      "        double sa = 0.0, sk = 0.0, sp = 0.0;\n        for (int64_t j = 0; j < n; ++j) {"),
    "diag_momentum_sign": ("p[d] += m[i] * vi[d];", "p[d] -= m[i] * vi[d];"),
    "diag_momentum_index": ("p[d] += m[i] * vi[d];", "p[d] += m[i] * vi[0];"),
    "diag_angmom_sign": ("l[2] += m[i] * (xi[0] * vi[1] - xi[1] * vi[0]);", "l[2] += m[i] * (xi[1] * vi[0] - xi[0] * vi[1]);"),
    "diag_kinetic_half": ("ke += 0.5 * m[i] *", "ke += m[i] *"),
    "pert_not_strict": ("if (m[j] / r2 > thr) {", "if (m[j] / r2 >= thr) {"),
    "pert_self_term": ("        int32_t found = 0;\n        for (int32_t s = 0; s < cap; ++s) lists[q * cap + s] = -1;\n        for (int64_t j = 0; j < n; ++j) {\n            if (j == i) continue;",
                       "        int32_t found = 0;\n        for (int32_t s = 0; s < cap; ++s) lists[q * cap + s] = -1;\n        for (int64_t j = 0; j < n; ++j) {"),
    "pert_no_softening": ("const double r2 = dx * dx + dy * dy + dz * dz + eps2;\n            if (m[j] / r2 > thr)",
                          "const double r2 = dx * dx + dy * dy + dz * dz;\n            if (m[j] / r2 > thr)"),
    "pert_mass_of_i": ("if (m[j] / r2 > thr) {", "if (m[i] / r2 > thr) {"),
    "pert_descending": ("        for (int64_t j = 0; j < n; ++j) {\n            if (j == i) continue;\n            const double dx = x[j] - x[i], dy = x[n + j] - x[n + i], dz = x[2 * n + j] - x[2 * n + i];\n            const double r2 = dx * dx + dy * dy + dz * dz + eps2;\n            if (m[j] / r2 > thr)",
                        "        for (int64_t j = n - 1; j >= 0; --j) {\n            if (j == i) continue;\n            const double dx = x[j] - x[i], dy = x[n + j] - x[n + i], dz = x[2 * n + j] - x[2 * n + i];\n            const double r2 = dx * dx + dy * dy + dz * dz + eps2;\n            if (m[j] / r2 > thr)"),
    "pert_cap_short": ("if (found < cap) lists[q * cap + found] = (int32_t)j;", "if (found < cap - 1) lists[q * cap + found] = (int32_t)j;"),
}

CHILD = r"""
import sys, traceback
sys.path.insert(0, {root!r})
import oracle
oracle.use_library({lib!r})
from tests import oracle_pins
failed = []
for pin in oracle_pins.ALL_PINS:
    try:
        pin()
    except Exception as e:
        failed.append(pin.__name__)
print("FAILED_PINS", failed)
sys.exit(0 if failed else 3)
"""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique/found"
    mutated = src.replace(old, new)
    csrc = tmp_path / "oracle_mut.c"
    csrc.write_text(mutated)
    lib = tmp_path / "liboracle_mut.so"
    sys.path.insert(0, ROOT)
    import oracle

    subprocess.run(["gcc", *oracle.CFLAGS, "-o", str(lib), str(csrc), "-lm"], check=True)
    env = dict(os.environ, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=str(lib))], cwd=ROOT,
                       capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, f"mutant {name} passed every pin:\n{r.stdout}\n{r.stderr}"
