"""Host-side: the surrogate file functions of the C ABI (no device call).
A written surrogate reads back bit for bit (configuration, parameters, Adam
state, bound table, predictor choice, counts); a damaged, truncated or
mismatched file is refused with the documented status."""
import numpy as np
import pytest

from paper_2410_05408_amd import gl


def arrays(seed=0):
    rng = np.random.default_rng(seed)
    n, nb = gl.gl_mlp_num_params(), gl.gl_surrogate_num_bins()
    cfg = gl.gl_surrogate_config_default()
    cfg.seed = int(rng.integers(1 << 40))
    cfg.epochs = 3
    p, m, v = (rng.standard_normal(n).astype(np.float32) for _ in range(3))
    t = rng.uniform(-1, 1, nb).astype(np.float32)
    z = (rng.uniform(size=nb) < 0.3).astype(np.uint8)
    c = rng.integers(0, 5000, nb).astype(np.int32)
    return cfg, p, m, v, 12345, t, z, c


def test_round_trip_is_exact(tmp_path):
    a = arrays()
    path = str(tmp_path / "s.glsur")
    gl.gl_surrogate_file_write(path, *a)
    b = gl.gl_surrogate_file_read(path)
    assert b[0].as_dict() == a[0].as_dict()
    for x, y in zip(a[1:], b[1:]):
        if isinstance(x, int):
            assert x == y
        else:
            assert np.asarray(x).tobytes() == np.asarray(y).tobytes()


def test_damaged_files_are_refused(tmp_path):
    a = arrays(2)
    path = tmp_path / "s.glsur"
    gl.gl_surrogate_file_write(str(path), *a)
    raw = path.read_bytes()
    cases = {
        "flipped payload byte": raw[:100] + bytes([raw[100] ^ 1]) + raw[101:],
        "flipped configuration byte": raw[:40] + bytes([raw[40] ^ 1]) + raw[41:],
        "truncated": raw[:-9],
        "trailing byte": raw + b"\0",
        "bad magic": b"X" + raw[1:],
        "old version": raw[:7] + b"1" + raw[8:],
        "empty": b"",
    }
    for name, data in cases.items():
        bad = tmp_path / "bad.glsur"
        bad.write_bytes(data)
        with pytest.raises(gl.GLError) as e:
            gl.gl_surrogate_file_read(str(bad))
        assert e.value.status == gl.GL_ERR_STATE, name
    with pytest.raises(gl.GLError) as e:
        gl.gl_surrogate_file_read(str(tmp_path / "missing.glsur"))
    assert e.value.status == gl.GL_ERR_STATE


def test_size_mismatches_and_nulls():
    import ctypes
    L = gl._sur_lib()
    cfg, p, m, v, step, t, z, c = arrays(3)
    fp, ft = gl._fptr(p), gl._fptr(t)
    zp, cp = gl._u8p(z), gl._i32p(c)
    assert L.gl_surrogate_file_write(b"/nonexistent/x", ctypes.byref(cfg), fp, fp, fp, 0, p.size - 1, ft, zp, cp,
                                     t.size) == gl.GL_ERR_SIZE
    assert L.gl_surrogate_file_write(b"/nonexistent/x", ctypes.byref(cfg), fp, fp, fp, 0, p.size, ft, zp, cp,
                                     t.size + 1) == gl.GL_ERR_SIZE
    assert L.gl_surrogate_file_write(None, ctypes.byref(cfg), fp, fp, fp, 0, p.size, ft, zp, cp,
                                     t.size) == gl.GL_ERR_NULL
    assert L.gl_surrogate_file_write(b"/nonexistent/x", ctypes.byref(cfg), fp, fp, fp, 0, p.size, ft, None, cp,
                                     t.size) == gl.GL_ERR_NULL
    assert L.gl_surrogate_file_write(b"/nonexistent/dir/x", ctypes.byref(cfg), fp, fp, fp, 0, p.size, ft, zp, cp,
                                     t.size) == gl.GL_ERR_STATE


def test_wrong_counts_in_header_are_size_errors(tmp_path):
    a = arrays(4)
    path = tmp_path / "s.glsur"
    gl.gl_surrogate_file_write(str(path), *a)
    raw = bytearray(path.read_bytes())
    raw[20:24] = (int.from_bytes(raw[20:24], "little") + 1).to_bytes(4, "little")  # n_params field
    path.write_bytes(bytes(raw))
    with pytest.raises(gl.GLError) as e:
        gl.gl_surrogate_file_read(str(path))
    assert e.value.status == gl.GL_ERR_SIZE


def test_default_configuration():
    c = gl.gl_surrogate_config_default()
    assert (c.n_train, c.n_calib, c.epochs, c.batch) == (20_000_000, 1_000_000, 4, 8192)
    assert c.safety == 4.0 and c.min_bin_count == 200 and c.zero_predictor == 0
