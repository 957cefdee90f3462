"""Host-side: the surrogate file functions of the C ABI (no device call).
A saved surrogate reads back bit for bit; a damaged, truncated or
mismatched file is refused with the documented status and leaves the
outputs untouched."""
import numpy as np
import pytest

from paper_2410_05408_amd import gl


def arrays(seed=0):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(gl.gl_mlp_num_params()).astype(np.float32)
    t = rng.uniform(-1, 1, gl.gl_surrogate_num_bins()).astype(np.float32)
    z = (rng.uniform(size=t.size) < 0.3).astype(np.uint8)
    return p, t, z


def test_round_trip_is_exact(tmp_path):
    p, t, z = arrays()
    path = str(tmp_path / "s.glsur")
    gl.gl_surrogate_save(path, p, t, z)
    p2, t2, z2 = gl.gl_surrogate_load(path)
    assert p2.tobytes() == p.tobytes() and t2.tobytes() == t.tobytes() and np.array_equal(z2, z)


def test_missing_choice_reads_back_as_zeros(tmp_path):
    p, t, _ = arrays(1)
    path = str(tmp_path / "s.glsur")
    gl.gl_surrogate_save(path, p, t, None)
    _, _, z2 = gl.gl_surrogate_load(path)
    assert not z2.any()


def test_damaged_files_are_refused(tmp_path):
    p, t, z = arrays(2)
    path = tmp_path / "s.glsur"
    gl.gl_surrogate_save(str(path), p, t, z)
    raw = path.read_bytes()
    cases = {
        "flipped payload byte": raw[:100] + bytes([raw[100] ^ 1]) + raw[101:],
        "truncated": raw[:-9],
        "trailing byte": raw + b"\0",
        "bad magic": b"X" + raw[1:],
        "empty": b"",
    }
    for name, data in cases.items():
        bad = tmp_path / "bad.glsur"
        bad.write_bytes(data)
        with pytest.raises(gl.GLError) as e:
            gl.gl_surrogate_load(str(bad))
        assert e.value.status == gl.GL_ERR_STATE, name
    with pytest.raises(gl.GLError) as e:
        gl.gl_surrogate_load(str(tmp_path / "missing.glsur"))
    assert e.value.status == gl.GL_ERR_STATE


def test_size_mismatches_and_nulls():
    L = gl._sur_lib()
    p, t, z = arrays(3)
    fp = gl._fptr(p)
    ft = gl._fptr(t)
    assert L.gl_surrogate_save(b"/nonexistent/x", fp, p.size - 1, ft, None, t.size) == gl.GL_ERR_SIZE
    assert L.gl_surrogate_save(b"/nonexistent/x", fp, p.size, ft, None, t.size + 1) == gl.GL_ERR_SIZE
    assert L.gl_surrogate_save(None, fp, p.size, ft, None, t.size) == gl.GL_ERR_NULL
    assert L.gl_surrogate_load(b"/nonexistent/x", None, p.size, ft, None, t.size) == gl.GL_ERR_NULL
    assert L.gl_surrogate_save(b"/nonexistent/dir/x", fp, p.size, ft, None, t.size) == gl.GL_ERR_STATE


def test_wrong_counts_in_header_are_size_errors(tmp_path):
    p, t, z = arrays(4)
    path = tmp_path / "s.glsur"
    gl.gl_surrogate_save(str(path), p, t, z)
    raw = bytearray(path.read_bytes())
    raw[20:24] = (int.from_bytes(raw[20:24], "little") + 1).to_bytes(4, "little")  # n_params field
    path.write_bytes(bytes(raw))
    with pytest.raises(gl.GLError) as e:
        gl.gl_surrogate_load(str(path))
    assert e.value.status == gl.GL_ERR_SIZE
