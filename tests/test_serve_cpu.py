"""Host logic of render serving (no GPU): the seeded request generator and
the slot-table layout shared with the packed kernel."""
import ctypes

import numpy as np


def _poses():
    from synth import cameras
    return [list(cameras.orbit_cams(seed=s, n=3)) for s in range(3)]


def test_requests_are_seeded_sorted_and_poisson():
    from paper_2305_13220_amd.serve import poisson_requests
    res = ((320, 240), (1920, 1080))
    a = poisson_requests(4000, qps=250.0, n_grids=3, cams_per_grid=_poses(), resolutions=res,
                         seed=[0, 5, 1])
    b = poisson_requests(4000, qps=250.0, n_grids=3, cams_per_grid=_poses(), resolutions=res,
                         seed=[0, 5, 1])
    assert [(r.grid, r.width, r.arrival) for r in a] == [(r.grid, r.width, r.arrival) for r in b]
    t = np.array([r.arrival for r in a])
    assert np.all(np.diff(t) > 0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    # exponential gaps: mean 1/qps, coefficient of variation 1
    assert abs(gaps.mean() * 250.0 - 1.0) < 0.05
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05
    assert {r.grid for r in a} == {0, 1, 2}
    assert {(r.width, r.height) for r in a} == set(res)


def test_request_intrinsics_follow_resolution():
    from paper_2305_13220_amd.serve import poisson_requests
    poses = _poses()
    for r in poisson_requests(50, qps=10.0, n_grids=3, cams_per_grid=poses,
                              resolutions=((640, 480), (1296, 968)), seed=3):
        f = (r.width / 2) / np.tan(np.deg2rad(30.0))
        np.testing.assert_allclose(r.cam[:4], [f, f, r.width / 2, r.height / 2], rtol=1e-6)
        # the pose part is one of the grid's poses, unchanged
        assert any(np.array_equal(r.cam[4:], np.asarray(p, np.float32)[4:]) for p in poses[r.grid])
        assert r.out_bytes(3) == r.width * r.height * 4 * 9


def test_slot_layout_matches_c_struct():
    from paper_2305_13220_amd.serve import SLOT_DTYPE, SlotC
    assert SLOT_DTYPE.itemsize == ctypes.sizeof(SlotC) == 136
    assert SLOT_DTYPE.fields["cam"][1] == SlotC.cam.offset == 32
    assert SLOT_DTYPE.fields["nsamples"][1] == SlotC.nsamples.offset == 128
