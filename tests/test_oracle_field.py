"""Pins of H(x, t): three independent routes agree, and the cell's symmetry holds."""
import numpy as np
from oracle import collocation, field, green, timegrid
from paper_2605_13987_amd import workloads


def _tiny():
    cfg = workloads.small_pixel(k=21, n_xy=8, n_z=16, n_freq=4, n_time=5, n_pairs=2, n_colloc=6)
    return cfg


def test_superposition_fft_and_column_routes_agree():
    cfg = _tiny()
    cell, cols, spec = cfg["cell"], cfg["columns"], cfg["spectrum"]
    s = green.smoothing_widths(cell, cols)
    sol = collocation.solve_spectrum(cell, cols, spec)
    qt = timegrid.to_time(sol["q"], spec)
    src = collocation.sources(cols)
    H2 = field.field_fft(cell, s, src, qt)
    pts = field.grid_points(cell)
    H1 = field.field_superposition(pts, cell, s, src, qt).reshape(H2.shape)
    scale = np.max(np.abs(H2))
    assert np.max(np.abs(H1 - H2)) <= 1e-12 * scale
    ij = [(0, 0), (3, 5), (7, 7), (4, 4)]
    H3 = field.field_columns(cell, s, src, qt, ij)
    for c, (i, j) in enumerate(ij):
        assert np.max(np.abs(H3[c] - H2[i, j])) <= 1e-12 * scale


def test_column_route_matches_fft_on_32x32x64(px32, px32_oracle):
    cell, cols = px32["cell"], px32["columns"]
    s = green.smoothing_widths(cell, cols)
    ij = [(0, 0), (16, 16), (5, 27), (31, 2)]
    H3 = field.field_columns(cell, s, px32_oracle["src"], px32_oracle["q_t"], ij)
    H = px32_oracle["H"]
    for c, (i, j) in enumerate(ij):
        assert np.max(np.abs(H3[c] - H[i, j])) <= 1e-11 * np.max(np.abs(H))


def test_c4_and_mirror_symmetry_about_the_readout(px32, px32_oracle):
    """Equal bias quarter-columns on a square cell: the axis charges are C4
    symmetric about the readout axis, hence so is H (as a vector field)."""
    H = px32_oracle["H"]
    N = px32["cell"]["N"][0]
    i = np.arange(N)
    # rotation (u, v) -> (-v, u) about the readout axis maps node (i, j) to (N - j, i)
    I, J = np.meshgrid(i, i, indexing="ij")
    Hx_rot = H[(N - J) % N, I, :, :, 0]
    Hy_rot = H[(N - J) % N, I, :, :, 1]
    Hz_rot = H[(N - J) % N, I, :, :, 2]
    sc = np.max(np.abs(H))
    assert np.max(np.abs(Hx_rot + H[I, J, :, :, 1])) <= 1e-12 * sc
    assert np.max(np.abs(Hy_rot - H[I, J, :, :, 0])) <= 1e-12 * sc
    assert np.max(np.abs(Hz_rot - H[I, J, :, :, 2])) <= 1e-12 * sc
    # mirror x -> p - x
    Hm = H[(N - i) % N]
    assert np.max(np.abs(Hm[..., 0] + H[..., 0])) <= 1e-12 * sc
    assert np.max(np.abs(Hm[..., 1:] - H[..., 1:])) <= 1e-12 * sc


def test_planar_fft_column_route_matches_the_other_routes(px32, px32_oracle):
    """The in-plane-FFT column route equals the direct column sums and the 3D
    FFT route, on a grid with both column axes (readout and corner bias)."""
    cell, cols = px32["cell"], px32["columns"]
    s = green.smoothing_widths(cell, cols)
    ij = [(0, 0), (16, 16), (5, 27), (31, 2), (17, 15), (0, 31)]
    H4 = field.field_columns_planar_fft(cell, s, px32_oracle["src"], px32_oracle["q_t"], ij, chunk=4)
    H3 = field.field_columns(cell, s, px32_oracle["src"], px32_oracle["q_t"], ij)
    H = px32_oracle["H"]
    sc = np.max(np.abs(H))
    assert np.max(np.abs(H4 - H3)) <= 1e-12 * sc
    for c, (i, j) in enumerate(ij):
        assert np.max(np.abs(H4[c] - H[i, j])) <= 1e-11 * sc


def test_planar_fft_column_route_on_an_anisotropic_grid():
    cfg = workloads.small_pixel(k=23, n_xy=12, n_z=20, n_freq=4, n_time=6, n_pairs=2, n_colloc=6)
    cell, cols, spec = cfg["cell"], cfg["columns"], cfg["spectrum"]
    s = green.smoothing_widths(cell, cols)
    sol = collocation.solve_spectrum(cell, cols, spec)
    qt = timegrid.to_time(sol["q"], spec)
    src = collocation.sources(cols)
    ij = [(i, j) for i in range(12) for j in range(0, 12, 5)]
    H4 = field.field_columns_planar_fft(cell, s, src, qt, ij, chunk=5)
    H3 = field.field_columns(cell, s, src, qt, ij)
    assert np.max(np.abs(H4 - H3)) <= 1e-12 * np.max(np.abs(H3))


def test_node_route_matches_the_column_routes(px32, px32_oracle):
    """The node-wise route equals the direct column sums and the 3D FFT route
    at scattered nodes (both column axes, every z residue, chunk edges)."""
    cell, cols = px32["cell"], px32["columns"]
    s = green.smoothing_widths(cell, cols)
    rng = np.random.default_rng(7)
    ix, iy, iz = rng.integers(0, 32, 300), rng.integers(0, 32, 300), rng.integers(0, 64, 300)
    ix[:3], iy[:3] = [0, 16, 31], [0, 16, 31]
    Hn = field.field_nodes_planar_fft(cell, s, px32_oracle["src"], px32_oracle["q_t"], ix, iy, iz, chunk=64)
    H = px32_oracle["H"]
    sc = np.max(np.abs(H))
    assert np.max(np.abs(Hn - H[ix, iy, iz])) <= 1e-11 * sc
    ij = [(0, 0), (16, 16), (5, 27)]
    H3 = field.field_columns(cell, s, px32_oracle["src"], px32_oracle["q_t"], ij)
    for c, (i, j) in enumerate(ij):
        z = np.arange(64)
        Hc = field.field_nodes_planar_fft(cell, s, px32_oracle["src"], px32_oracle["q_t"], np.full(64, i),
                                          np.full(64, j), z)
        assert np.max(np.abs(Hc - H3[c])) <= 1e-12 * sc


def test_node_route_on_an_anisotropic_grid():
    cfg = workloads.small_pixel(k=29, n_xy=12, n_z=20, n_freq=4, n_time=6, n_pairs=2, n_colloc=6)
    cell, cols, spec = cfg["cell"], cfg["columns"], cfg["spectrum"]
    s = green.smoothing_widths(cell, cols)
    sol = collocation.solve_spectrum(cell, cols, spec)
    qt = timegrid.to_time(sol["q"], spec)
    src = collocation.sources(cols)
    ij = [(i, j) for i in range(12) for j in range(0, 12, 5)]
    H3 = field.field_columns(cell, s, src, qt, ij)
    ix = np.repeat([i for i, _ in ij], 20)
    iy = np.repeat([j for _, j in ij], 20)
    iz = np.tile(np.arange(20), len(ij))
    Hn = field.field_nodes_planar_fft(cell, s, src, qt, ix, iy, iz, chunk=37)
    assert np.max(np.abs(Hn.reshape(len(ij), 20, 6, 3) - H3)) <= 1e-12 * np.max(np.abs(H3))


def test_node_route_with_axes_off_the_symmetric_nodes():
    """Column axes shifted off the cell's symmetric nodes, so that a wrong
    sign of the in-plane shift or a swapped axis would show."""
    cfg = workloads.small_pixel(k=31, n_xy=12, n_z=20, n_freq=4, n_time=6, n_pairs=2, n_colloc=6)
    cell, spec = cfg["cell"], cfg["spectrum"]
    h = cell["L"][0] / cell["N"][0]
    cols = [dict(c, x=c["x"] + 3 * h, y=c["y"] + 1 * h) for c in cfg["columns"]]
    s = green.smoothing_widths(cell, cols)
    sol = collocation.solve_spectrum(cell, cols, spec)
    qt = timegrid.to_time(sol["q"], spec)
    src = collocation.sources(cols)
    ij = [(1, 2), (4, 1), (9, 7), (11, 0)]
    H3 = field.field_columns(cell, s, src, qt, ij)
    ix = np.repeat([i for i, _ in ij], 20)
    iy = np.repeat([j for _, j in ij], 20)
    iz = np.tile(np.arange(20), len(ij))
    Hn = field.field_nodes_planar_fft(cell, s, src, qt, ix, iy, iz)
    assert np.max(np.abs(Hn.reshape(len(ij), 20, 6, 3) - H3)) <= 1e-12 * np.max(np.abs(H3))
    H4 = field.field_columns_planar_fft(cell, s, src, qt, ij)
    assert np.max(np.abs(H4 - H3)) <= 1e-12 * np.max(np.abs(H3))
