"""C-ABI checks that need no GPU: the library loads, exports every declared entry point,
and rejects invalid fibre descriptions before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2401_18022_amd import binding as B
from paper_2401_18022_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "isrsgn.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(isrsgn_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = C.CDLL(B.LIB_PATH)
    syms = declared_symbols()
    assert set(B.SYMBOLS) == set(syms), "binding and header disagree"
    for s in syms:
        assert hasattr(L, s), s


def _setup(**kw):
    fb = W.tiny_fibre().replace(**kw)
    d, keep = B.make_desc(fb)
    h = C.c_void_p()
    rc = B.lib().isrsgn_setup_fibre(C.byref(d), C.byref(h))
    return rc, h, B.lib().isrsgn_last_error().decode()


@pytest.mark.parametrize("kw, needle", [
    (dict(span_m=0.0), "span_m"),
    (dict(n_steps=0), "n_steps"),
    (dict(grid_s=1), "grid_s"),
    (dict(grid_v=1), "grid_v"),
    (dict(grid_s=5000), "grid_s"),
    (dict(s_decades=0.0), "s_decades"),
    (dict(ode_sub=0), "ode_sub"),
    (dict(n_spans=0), "n_spans"),
    (dict(precision=7), "precision"),
    (dict(profile=9), "profile"),
    (dict(beta2=float("nan")), "finite"),
])
def test_setup_rejects_invalid_descriptions(kw, needle):
    rc, h, msg = _setup(**kw)
    assert rc in (B.ISRSGN_EINVAL, B.ISRSGN_EUNSUPPORTED)
    assert needle in msg
    assert not h.value


def test_closed_form_needs_uniform_fibre():
    fb = W.cl_fibre().replace(profile=W.PROFILE_CLOSED_FORM)
    d, keep = B.make_desc(fb)
    h = C.c_void_p()
    assert B.lib().isrsgn_setup_fibre(C.byref(d), C.byref(h)) == B.ISRSGN_EINVAL
    assert "n_tab" in B.lib().isrsgn_last_error().decode()


def test_unsorted_table_rejected():
    fb = W.cl_fibre()
    fb = fb.replace(tab_f_hz=fb.tab_f_hz[::-1].copy())
    d, keep = B.make_desc(fb)
    h = C.c_void_p()
    assert B.lib().isrsgn_setup_fibre(C.byref(d), C.byref(h)) == B.ISRSGN_EINVAL


def test_null_arguments_and_destroy_null():
    L = B.lib()
    assert L.isrsgn_setup_fibre(None, None) == B.ISRSGN_EINVAL
    assert L.isrsgn_eta(None, None, None, None, None, None, None) == B.ISRSGN_EINVAL
    assert L.isrsgn_snr(None, None, None, None, 0.0, None, None, None) == B.ISRSGN_EINVAL
    assert L.isrsgn_snr_grad(None, None, None, None, 0.0, None, None, None, None) == B.ISRSGN_EINVAL
    assert L.isrsgn_profile(None, None, None, None, None, None, None, None) == B.ISRSGN_EINVAL
    assert L.isrsgn_set_timing(None, 1) == B.ISRSGN_EINVAL
    assert L.isrsgn_set_checks(None, 1) == B.ISRSGN_EINVAL
    assert L.isrsgn_stage_times(None, None, 0) == B.ISRSGN_EINVAL
    L.isrsgn_destroy(None)
    assert isinstance(L.isrsgn_last_error(), bytes)


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2401_18022_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                for bad in ("import oracle", "from oracle", "liboracle", "orc_"):
                    assert bad not in text, (f, bad)


def test_segment_counts_reproduce_table2():
    """N_B = round(B_band / B_p), B_band = channels x 100 GHz, B_p = 750 GHz (O) / 1.5 THz (Sec. IV):
    the paper's channel counts give its segment counts (Table II)."""
    import json
    from paper_2401_18022_amd import optimise
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "table2_noise_figure.json")))
    assert optimise.segment_counts(g["channels"]) == g["segments"]
    assert sum(g["segments"]) == 49


def test_segment_matrix_interpolates():
    from paper_2401_18022_amd import optimise
    f = W.ou_grid()
    A, counts = optimise.segment_matrix(f)
    np.testing.assert_allclose(A.sum(1), 1.0, rtol=1e-12)    # partition of unity per channel
    x = np.linspace(-5, 5, A.shape[1])
    p = A @ x
    assert p.min() >= -5 - 1e-12 and p.max() <= 5 + 1e-12
    assert A.shape == (589, sum(counts)) and all(c >= 2 for c in counts)
