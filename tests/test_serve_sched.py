"""Host logic of the streaming server: ring slots, scheduling order, overwrite
safety and HBM admission, simulated on the CPU with frame indices standing in
for frames (no device)."""
import numpy as np
import pytest

from paper_2004_00923_amd.serve import (AdmissionError, Admission, CameraSpec, CamState, RingPlan, Scheduler,
                                        camera_bytes)


def _simulate(specs, targets, arrivals, max_batch=16, per_camera=2):
    """Run the scheduler against simulated rings.  specs: [(window, hop)];
    arrivals: list of per-pass available-frame counts.  Checks every copy only
    overwrites a transformed frame and every analysed window holds its frames in
    order.  Returns the analysed batches."""
    states = [CamState(RingPlan(w, h), t) for (w, h), t in zip(specs, targets)]
    sched = Scheduler(states, max_batch, per_camera)
    u16 = [np.full(s.ring.R, -1) for s in states]
    holo = [np.full(s.ring.slots, -1) for s in states]
    transformed = [set() for _ in states]
    batches = []
    for avail in arrivals:
        for a in sched.step(avail):
            if a[0] == "copy":
                _, i, lo, hi = a
                for k in range(lo, hi):
                    s = states[i].ring.slot(k)
                    assert u16[i][s] == -1 or u16[i][s] in transformed[i], "frame overwritten before its transform"
                    u16[i][s] = k
            elif a[0] == "fresnel":
                _, i, runs = a
                for src, dst, n in runs:
                    assert dst + n <= states[i].ring.slots and src + n <= states[i].ring.R
                    holo[i][dst:dst + n] = u16[i][src:src + n]
                    transformed[i].update(u16[i][src:src + n].tolist())
            else:
                assert len(a[1]) <= max_batch
                for i, c in a[1]:
                    r = states[i].ring
                    s = r.window_slot(c)
                    want = np.arange(c * r.hop, c * r.hop + r.window)
                    assert np.array_equal(holo[i][s:s + r.window], want), f"camera {i} window {c}"
                batches.append(list(a[1]))
        if all(s.done() for s in states):
            break
    return states, batches


@pytest.mark.parametrize("window,hop", [(32, 25), (32, 32), (32, 1), (32, 8), (16, 40), (3, 2)])
def test_ring_windows_contiguous_and_ordered(window, hop):
    r = RingPlan(window, hop)
    assert r.R % hop == 0 and r.R >= window
    for c in range(200):
        s = r.window_slot(c)
        assert s + window <= r.slots
    # a frame copied into slot s < M is also written to R + s
    runs = r.fresnel_runs(0, 3 * r.R)
    covered = sorted((d, n) for _, d, n in runs)
    assert sum(n for _, n in covered) == 3 * r.R + 3 * min(r.M, r.R)


@pytest.mark.parametrize("window,hop", [(32, 25), (32, 16), (32, 1), (16, 40)])
def test_scheduler_unthrottled_single_camera(window, hop):
    st, batches = _simulate([(window, hop)], [12], [[10 ** 9]] * 400)
    assert st[0].done()
    order = [c for b in batches for _, c in b]
    assert order == list(range(12))


def test_scheduler_paced_two_cameras_batches_across_cameras():
    # camera 0 at twice the frame rate of camera 1; passes every 20 frame periods of camera 0
    specs = [(32, 25), (32, 25)]
    arrivals = [[20 * t, (20 * t) // 2] for t in range(1, 400)]
    st, batches = _simulate(specs, [14, 7], arrivals)
    assert all(s.done() for s in st)
    for cam in (0, 1):
        assert [c for b in batches for i, c in b if i == cam] == list(range([14, 7][cam]))
    assert any(len({i for i, _ in b}) == 2 for b in batches), "no batch mixed the two cameras"


def test_scheduler_late_host_respects_ring_and_batch_limits():
    # the host falls behind: everything arrives at once; the ring admits at most R
    # frames beyond the oldest pending window, batches hold <= per_camera windows per camera
    st, batches = _simulate([(32, 25), (32, 8)], [9, 20], [[10 ** 6, 10 ** 6]] * 200, max_batch=3, per_camera=2)
    assert all(s.done() for s in st)
    for b in batches:
        assert len(b) <= 3
        for cam in (0, 1):
            assert sum(1 for i, _ in b if i == cam) <= 2


def test_scheduler_no_windows_before_first_full_window():
    st, batches = _simulate([(32, 25)], [1], [[31]] * 5)
    assert batches == [] and not st[0].done()


def test_admission_budget():
    a = CameraSpec("A", 1024, 1024, 500.0, 100)
    b = CameraSpec("B", 1024, 2048, 250.0, 101)
    ra, rb = RingPlan(32, 25), RingPlan(32, 25)
    need_a = sum(camera_bytes(a, ra, 4).values())
    need_b = sum(camera_bytes(b, rb, 4).values())
    # the hologram ring dominates: (R + M) frames of complex64
    assert camera_bytes(a, ra, 4)["holo"] == (50 + 7) * 1024 * 1024 * 8
    assert need_b > need_a
    adm = Admission(need_a + need_b)
    adm.request(a, ra)
    adm.request(b, rb)
    assert adm.used == need_a + need_b
    small = Admission(need_a + need_b - 1)
    small.request(a, ra)
    with pytest.raises(AdmissionError):
        small.request(b, rb)
    assert small.used == need_a      # a rejected camera takes nothing
    with pytest.raises(AdmissionError):
        Admission(need_a - 1).request(a, ra)
