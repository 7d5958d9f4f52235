"""The C-ABI library loads and exports every entry point include/ire.h declares
(host-only checks: nothing here launches GPU work)."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:ire|sur)_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2408_13807_amd import ire
    lib = ire.library()
    names = declared("ire.h")
    assert len(names) >= 18
    for name in names:
        assert hasattr(lib, name), name
    from paper_2408_13807_amd import surrogate
    assert sorted(ire.EXPORTS + surrogate.EXPORTS) == names


def test_options_layout_and_defaults():
    from paper_2408_13807_amd import ire
    o = ire.default_options()
    assert (o.k_bg, o.ffi, o.w_floor, o.max_events, o.stepping, o.max_lanes, o.reemit_uniform,
            o.aggregate, o.batch) == (0.5, 0, 1e-10, 1000000, 0, 0, 0, -1, 0)
    assert (o.use_g_E, o.g_E, o.use_g_S, o.g_S, o.k_A, o.k_S) == (0, 0.0, 0, 0.0, 1.0, 1.0)
    assert (o.k_A_rho, o.k_A_lowest, o.k_A_highest, o.replicas, o.quorum) == (0, 3.0, 1.0, 1, 0)
    b = ire.default_batch_options()
    assert (b.use_g_E, b.g_E, b.use_g_S, b.g_S, b.k_A, b.k_S, b.use_graph) == (0, 0.0, 0, 0.0, 1.0, 1.0, 1)


def test_planck_helper_matches_oracle(orc):
    from paper_2408_13807_amd import ire
    nu = np.geomspace(1e10, 1e16, 50)
    for T in (3.0, 20.0, 5000.0):
        got = ire.planck(nu, T)
        want = np.array([orc.planck(x, T) for x in nu])
        np.testing.assert_allclose(got, want, rtol=1e-13, atol=0)


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2408_13807_amd import ire
    with pytest.raises(ire.IREError) as e:
        ire.IREModel(0)
    assert e.value.code == ire.IRE_E_DEVICE


def test_null_handle_calls_are_safe():
    from paper_2408_13807_amd import ire
    lib = ire.library()
    lib.ire_destroy(None)
    assert lib.ire_set_options(None, None) == ire.IRE_E_INVALID
    assert lib.ire_run(None, 1, 0, 1, None) == ire.IRE_E_INVALID
    assert lib.ire_last_error(None) == b"null handle"


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C compiler's field
    offsets and sizes (a field added on one side only fails here)."""
    from paper_2408_13807_amd import ire, surrogate
    pairs = [("ire_options", ire.Options), ("ire_stats", ire.Stats), ("ire_model_desc", ire.ModelDesc),
             ("ire_batch_options", ire.BatchOptions), ("ire_batch_stats", ire.BatchStats),
             ("sur_train_opts", surrogate.TrainOpts)]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "ire.h"', "int main(void) {"]
    for cname, py in pairs:
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {(a, b): int(c) for a, b, c in (l.split() for l in out if l)}
    for cname, py in pairs:
        assert got[(cname, "sizeof")] == ct.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
