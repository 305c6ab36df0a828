"""Planted mistakes in the 2-D oracle must each fail a pin.

Each case below edits one step of ``oracle/rt_oracle.c`` into a plausible
mistake (the kind a reader checking the oracle against the paper could miss),
compiles the edited copy on the CPU, and runs the oracle's 2-D pins against
it.  At least one pin must fail for every case: otherwise the pins would not
tell that implementation from the correct one.  The unedited oracle passes
every pin in the regular test run.

Steps covered: the (ln r, z/r) index map and bilinear fetch (O4, O5), the
border taper (S5), the surfaces' interpolation and the logistic CO mask (S6),
the LTE populations and the march (O6, O8).
"""
import os

import pytest

import oracle
from oracle import build as obuild

import test_oracle_fetch_pins as F
import test_oracle_pins as P

# the 2-D border taper, as the oracle writes it
TAPER = ("const double taper = clampd(u + 1.0, 0.0, 1.0) * clampd(P->nr - u, 0.0, 1.0) * "
         "clampd(P->nz - v, 0.0, 1.0);")

# (what the mistake is, text of the correct step, text of the mistake)
MUTANTS = [
    ("density interpolated linearly instead of its logarithm",
     "const double ln_n = BIL(P->ln_nh2);",
     "const double ln_n = log(w00 * exp((double)P->ln_nh2[n00]) + w01 * exp((double)P->ln_nh2[n01])"
     " + w10 * exp((double)P->ln_nh2[n10]) + w11 * exp((double)P->ln_nh2[n11]));"),
    ("radial and vertical bilinear weights swapped",
     "const double fu = uc - i0, fv = vc - j0;",
     "const double fu = vc - j0, fv = uc - i0;"),
    ("radial index linear in r instead of ln r",
     "const double u = log(rho / P->r_min_au) / dln;",
     "const double u = (rho - P->r_min_au) / (P->r_max_au - P->r_min_au) * (P->nr - 1);"),
    ("vertical index from z over the spherical radius",
     "const double v = (a / rho) / dzr;",
     "const double v = (a / sqrt(rho * rho + a * a)) / dzr;"),
    ("mask width uses the log-radius spacing",
     "const double w = P->mask_width * rho * dzr;",
     "const double w = P->mask_width * rho * dln;"),
    ("mask width without the radius",
     "const double w = P->mask_width * rho * dzr;",
     "const double w = P->mask_width * dzr;"),
    ("upper-surface logistic with its sign flipped",
     "sigm((zup - a) / w)",
     "sigm((a - zup) / w)"),
    ("surfaces interpolated with the vertical weight",
     "double zlo = (1 - fu) * (double)P->z_lo_au[i0] + fu * (double)P->z_lo_au[i0 + 1];",
     "double zlo = (1 - fv) * (double)P->z_lo_au[i0] + fv * (double)P->z_lo_au[i0 + 1];"),
    ("outer taper starts one cell inside the grid",
     TAPER, TAPER.replace("clampd(P->nr - u,", "clampd(P->nr - 1.0 - u,")),
    ("inner taper two cells long",
     TAPER, TAPER.replace("clampd(u + 1.0,", "clampd(0.5 * (u + 2.0),")),
    ("vertical taper missing",
     TAPER, TAPER.replace(" * clampd(P->nz - v, 0.0, 1.0);", ";")),
    ("fetch clamps the vertical index one node short",
     "vc = clampd(v, 0.0, P->nz - 1);",
     "vc = clampd(v, 0.0, P->nz - 2);"),
]


def _pins():
    """The 2-D pins, as (name, call) pairs."""
    out = []
    for name in dir(F):
        fn = getattr(F, name)
        if name.startswith("test_") and callable(fn):
            if name == "test_mask_width_and_lower_surface":
                out += [(f"{name}[{w}]", (lambda fn=fn, w=w: fn(w))) for w in (1.0, 2.5)]
            else:
                out.append((name, fn))
    out.append(("isothermal_slab", lambda: P.test_isothermal_slab(40.0, 13.815510557964274)))
    out += [(n, getattr(P, n)) for n in ("test_optically_thin_limit", "test_source_function_is_planck",
                                          "test_thin_ring_doppler_sign", "test_bounds_and_zero_density",
                                          "test_recurrence_equals_nested_sum")]
    return out


@pytest.mark.parametrize("what,good,bad", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(what, good, bad, tmp_path, monkeypatch):
    with open(obuild.SRC) as fh:
        src = fh.read()
    assert src.count(good) == 1, f"the step to edit is not in the oracle as expected: {good!r}"
    mutant = os.path.join(tmp_path, "rt_oracle_mutant.c")
    with open(mutant, "w") as fh:
        fh.write(src.replace(good, bad))
    so = obuild.build(src=mutant, out=os.path.join(tmp_path, "librt_oracle_mutant.so"))
    monkeypatch.setattr(oracle, "_lib", oracle.load(so))
    failed = []
    for name, fn in _pins():
        try:
            fn()
        except (AssertionError, ArithmeticError, ValueError):
            failed.append(name)
    assert failed, f"no pin fails when the oracle has this mistake: {what}"
