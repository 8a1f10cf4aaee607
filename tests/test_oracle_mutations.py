"""The oracle's pins catch plausible mistakes.

Each case copies oracle.c, plants one mistake by a textual substitution,
compiles the copy on the CPU and runs pins from test_oracle.py against it;
at least one of the named pins must fail.  Nothing here touches a GPU."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle as P

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTATIONS = [
    # (name, original text, planted text, pins that must catch it)
    ("displacement sign", "double dx = x[j] - x[p];", "double dx = x[p] - x[j];",
     [P.test_two_body_closed_form]),
    ("power of r", "double s = G * mass[j] / (r2 * r);\n        cs_add",
     "double s = G * mass[j] / (r2 * r2);\n        cs_add", [P.test_two_body_closed_form]),
    ("source mass index", "double s = G * mass[j] / (r2 * r);\n        cs_add",
     "double s = G * mass[p] / (r2 * r);\n        cs_add", [P.test_two_body_closed_form]),
    ("self pair kept", "        if (j == p) continue;\n        double dx = x[j] - x[p];",
     "        double dx = x[j] - x[p];", [P.test_two_body_closed_form]),
    ("dropped 1/2 in the drift", "pos[k] + vel[k] * dt + 0.5 * a0[k] * dt * dt",
     "pos[k] + vel[k] * dt + a0[k] * dt * dt",
     [lambda: P.test_circular_orbit_closes_with_second_order_error()]),
    ("velocity from the new acceleration only", "vel[k] + 0.5 * (a0[k] + a1[k]) * dt",
     "vel[k] + a1[k] * dt", [lambda: P.test_circular_orbit_closes_with_second_order_error()]),
    ("pairs counted twice in the potential", "for (int64_t j = i + 1; j < n; ++j) {",
     "for (int64_t j = 0; j < n; ++j) {\n            if (j == i) continue;",
     [P.test_energy_closed_form_circular]),
    ("angular momentum sign", "cs_add(&l[0], m * (ry * vz - rz * vy));",
     "cs_add(&l[0], m * (ry * vz + rz * vy));", [P.test_momenta_conserved]),
    ("diagonal Jacobian block sign",
     "o[a] -= G * mass[j] * (k[3 * a + 0] * uq[0]", "o[a] += G * mass[j] * (k[3 * a + 0] * uq[0]",
     [P.test_vjp_invariants, P.test_vjp_against_complex_step_jvp]),
    ("tidal tensor factor", "k[3 * a + b] = (a == b ? i3 : 0.0) - 3.0 * d[a] * d[b] * i5;",
     "k[3 * a + b] = (a == b ? i3 : 0.0) - 2.0 * d[a] * d[b] * i5;",
     [P.test_vjp_against_complex_step_jvp]),
    ("adjoint kick weight", "for (int64_t k = 0; k < m; ++k) ab[k] += 0.5 * dt * vb[k];",
     "for (int64_t k = 0; k < m; ++k) ab[k] += dt * vb[k];",
     [P.test_adjoint_dot_product_with_tangent]),
    ("adjoint drift", "vb[k] = vb[k] + dt * rb[k];", "vb[k] = vb[k] + 0.5 * dt * rb[k];",
     [P.test_adjoint_dot_product_with_tangent]),
    ("dual-number quotient rule", "(a.d * b.v - a.v * b.d) / (b.v * b.v)",
     "(a.d * b.v + a.v * b.d) / (b.v * b.v)", [P.test_tangent_against_finite_differences]),
    ("RK4 stage weight", "(kr1[k] + 2.0 * kr2[k] + 2.0 * kr3[k] + kr4[k])",
     "(kr1[k] + 1.0 * kr2[k] + 2.0 * kr3[k] + kr4[k])",
     [P.test_rk4_circular_orbit_fourth_order, P.test_rk4_eccentric_orbit_against_kepler]),
    ("RK4 third-stage position", "rs[k] = pos[k] + 0.5 * dt * kr2[k];",
     "rs[k] = pos[k] + 0.5 * dt * kr1[k];",
     [P.test_rk4_circular_orbit_fourth_order, P.test_rk4_eccentric_orbit_against_kepler]),
    ("RK4 last-stage velocity", "kr4[k] = vel[k] + dt * kv3[k];",
     "kr4[k] = vel[k] + 0.5 * dt * kv3[k];",
     [P.test_rk4_circular_orbit_fourth_order, P.test_rk4_eccentric_orbit_against_kepler]),
]


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert old in src, f"mutation anchor not found: {name}"
    path = tmp_path / "mut.c"
    path.write_text(src.replace(old, new, 1))
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared",
                    "-o", str(lib), str(path), "-lm"], check=True)
    return str(lib)


def _fails(pin):
    try:
        with np.errstate(all="ignore"):
            pin()
    except (AssertionError, ValueError, FloatingPointError, MemoryError):
        return True
    return False


@pytest.mark.parametrize("name,old,new,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, old, new, pins):
    lib = _build(tmp_path, name, old, new)
    with oracle.use_library(lib):
        caught = [_fails(pin) for pin in pins]
    assert any(caught), f"no pin caught the planted mistake '{name}'"


def test_unmutated_copy_passes(tmp_path):
    """Control: the same machinery with no change passes the same pins."""
    lib = _build(tmp_path, "none", "double dx = x[j] - x[p];", "double dx = x[j] - x[p];")
    with oracle.use_library(lib):
        for pin in (P.test_two_body_closed_form, P.test_energy_closed_form_circular,
                    P.test_vjp_invariants, P.test_adjoint_dot_product_with_tangent):
            pin()
