"""Host-side parts of the learned cost model (no GPU): the saved model file
round-trips every field training needs to resume, and holds only plain
arrays."""
import numpy as np

from paper_2311_12519_amd import costmodel as cm


def test_mlp_save_load_round_trip(tmp_path):
    m = cm.MLP(seed=3, device="cpu")
    m.mu = np.arange(8, dtype=np.float64)
    m.sd = np.linspace(1, 2, 8)
    m.y_mu = -0.75
    m.m += 0.5
    m.v += 0.25
    m.step = 1234
    path = str(tmp_path / "model.npz")
    m.save(path)
    r = cm.MLP.load(path, device="cpu")
    assert np.array_equal(r.theta.numpy(), m.theta.numpy())
    assert np.array_equal(r.m.numpy(), m.m.numpy()) and np.array_equal(r.v.numpy(), m.v.numpy())
    assert r.step == 1234 and r.y_mu == -0.75
    assert np.array_equal(r.mu, m.mu) and np.array_equal(r.sd, m.sd)
    # plain arrays only: loadable without unpickling
    z = np.load(path, allow_pickle=False)
    assert set(z.files) == {"theta", "m", "v", "step", "mu", "sd", "y_mu"}
