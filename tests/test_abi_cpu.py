"""Host-side checks of the C ABI library: it loads without a GPU and exports
every entry point that include/gl.h declares.  No compute call is made."""
import os
import re

from paper_2410_05408_amd import gl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "gl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gl_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = gl.lib()
    names = declared_symbols()
    assert "gl_lightcurve_batch" in names and len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(gl.EXPORTED)


def test_version_string():
    assert gl.gl_version() == "0.1.0"


def test_null_context_errors_without_device():
    L = gl.lib()
    # host-checkable errors return before touching any device
    assert L.gl_lightcurve_batch(None, None, 1, None, None, 1, None, None, None, None) == gl.GL_ERR_NULL
    assert L.gl_ctx_sync_status(None) == gl.GL_ERR_NULL
    assert L.gl_ctx_set_plan(None, 8) == gl.GL_ERR_NULL
    assert L.gl_ctx_last_error(None) == b"null context"


def test_flop_model_is_host_only():
    m = gl.gl_flop_model()
    assert m["gk21_pieces"] == 21 * 64 + 10
    assert m["trapezoid_nodes"] == 24
    assert m["sub_in_window"] > 0 and m["off_star_in_window"] == 0
