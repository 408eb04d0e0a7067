"""Reading series and designs from files (CPU only): formats, checks and the
lambda grid of the command-line front end."""
import numpy as np
import pytest

from paper_1808_06992_amd import ingest, synth


def test_load_formats_round_trip(tmp_path):
    rng = np.random.default_rng(0)
    s = rng.standard_normal((50, 4))
    np.save(tmp_path / "a.npy", s)
    np.savez(tmp_path / "b.npz", rec=s)
    np.savez(tmp_path / "c.npz", rec=s, other=s[:3])
    np.savetxt(tmp_path / "d.csv", s, delimiter=",")
    np.savetxt(tmp_path / "e.txt", s)
    assert np.array_equal(ingest.load_series(str(tmp_path / "a.npy")), s)
    assert np.array_equal(ingest.load_series(str(tmp_path / "b.npz")), s)
    assert np.array_equal(ingest.load_series(str(tmp_path / "c.npz"), "rec"), s)
    np.testing.assert_allclose(ingest.load_series(str(tmp_path / "d.csv")), s, rtol=1e-15)
    np.testing.assert_allclose(ingest.load_series(str(tmp_path / "e.txt")), s, rtol=1e-15)
    np.save(tmp_path / "t.npy", s.T)
    assert np.array_equal(ingest.load_series(str(tmp_path / "t.npy"), time_axis=1), s)


def test_load_rejects_bad_inputs(tmp_path):
    s = np.ones((10, 3))
    s[2, 1] = np.nan
    np.save(tmp_path / "nan.npy", s)
    with pytest.raises(ValueError, match="NaN"):
        ingest.load_series(str(tmp_path / "nan.npy"))
    np.save(tmp_path / "short.npy", np.ones((3, 2)))
    with pytest.raises(ValueError, match="too few"):
        ingest.load_series(str(tmp_path / "short.npy"), order=2)
    np.savez(tmp_path / "two.npz", a=np.ones(3), b=np.ones(3))
    with pytest.raises(ValueError, match="name the array"):
        ingest.load_array(str(tmp_path / "two.npz"))
    np.save(tmp_path / "obj.npy", np.array([{"a": 1}], dtype=object), allow_pickle=True)
    with pytest.raises(ValueError):
        ingest.load_array(str(tmp_path / "obj.npy"))       # never unpickled
    with pytest.raises(ValueError, match="unsupported"):
        ingest.load_array(str(tmp_path / "x.h5"))


def test_lambda_grid_matches_generator():
    pr = synth.var_d(6, 300, 2, 0.3, 0.8, 1, mu_scale=1.0, intercept=True, q=7)
    lam = ingest.lambda_grid(ingest._var_lambda_max(pr.series, 2, True), 7, 1e-3)
    np.testing.assert_allclose(lam, pr.lambdas, rtol=1e-12)
