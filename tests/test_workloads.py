"""The seeded input generators: the torch polyline stepper against the numpy
one, and the shape of the 256x256x512 workload."""
import numpy as np
import torch

from paper_2605_13987_amd import workloads


def test_torch_drift_matches_numpy_drift_without_diffusion():
    cfg = workloads.small_pixel(k=71, n_xy=16, n_z=32, n_freq=4, n_time=60, n_pairs=40, n_colloc=8)
    pos = cfg["carriers"]["pos"]
    q = cfg["carriers"]["charge"]
    ref = workloads.drift_paths(pos[:, 0], q, cfg["columns"], cfg["cell"], 60, 10e-12)
    got = workloads.drift_paths_torch(pos[:, 0], q, cfg["columns"], cfg["cell"], 60, 10e-12).numpy()
    assert np.max(np.abs(got - ref)) <= 1e-18


def test_diffusion_is_seeded_and_absorbs_on_the_surface():
    cfg = workloads.small_pixel(k=72, n_xy=16, n_z=32, n_freq=4, n_time=80, n_pairs=30, n_colloc=8)
    st, q = cfg["carriers"]["pos"][:, 0], cfg["carriers"]["charge"]
    a = workloads.drift_paths_torch(st, q, cfg["columns"], cfg["cell"], 80, 10e-12, diffusion_sigma=0.5e-6, seed=3)
    b = workloads.drift_paths_torch(st, q, cfg["columns"], cfg["cell"], 80, 10e-12, diffusion_sigma=0.5e-6, seed=3)
    c = workloads.drift_paths_torch(st, q, cfg["columns"], cfg["cell"], 80, 10e-12, diffusion_sigma=0.5e-6, seed=4)
    assert torch.equal(a, b) and not torch.equal(a, c)
    d = (a[:, 1:] - a[:, :-1]).numpy()
    moving = np.any(d != 0, axis=2)
    # once a carrier stops it stays put
    for row in moving:
        k = np.nonzero(~row)[0]
        if k.size:
            assert not row[k[0]:].any()
    # stopped carriers sit on their target column's surface, or short of it by
    # what the diffusion kick of their last step carried them (the stop is
    # taken along the drift direction)
    L = cfg["cell"]["L"]
    end = a[:, -1].numpy()
    stopped = ~moving[:, -1]
    assert stopped.sum() > 0
    for i in np.nonzero(stopped)[0]:
        col = cfg["columns"][0] if q[i] < 0 else cfg["columns"][1]
        _, dist = workloads.nearest_axis_point(end[i:i + 1], workloads._segments([col], cfg["cell"])[0], L)
        assert col["radius"] - 1e-12 <= dist[0] <= col["radius"] + 6 * 0.5e-6


def test_256x256x512_workload_shape():
    cfg = workloads.pixel_256x256x512_tracks(device="cpu", n_tracks=2, n_pairs=50)
    car = cfg["carriers"]
    assert cfg["cell"]["N"] == (256, 256, 512)
    assert cfg["spectrum"]["n_freq"] == 512 and cfg["spectrum"]["n_time"] == 400
    assert tuple(car["pos"].shape) == (200, 401, 3)
    assert sorted(set(car["track"].tolist())) == [0, 1] and car["n_tracks"] == 2
    assert abs(float(car["charge"].sum())) < 1e-30
