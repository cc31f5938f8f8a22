"""Host logic of the streaming server: ring slots, scheduling order, overwrite
safety and HBM admission, simulated on the CPU with frame indices standing in
for frames (no device)."""
import numpy as np
import pytest

from paper_2004_00923_amd.serve import (AdmissionError, Admission, CameraSpec, CamState, RingPlan, Scheduler,
                                        camera_bytes)


def _simulate(specs, targets, arrivals, max_batch=16, per_camera=2, missing=None, queue_caps=None):
    """Run the scheduler against simulated rings.  specs: [(window, hop)];
    arrivals: list of per-pass available-frame counts.  Checks every copy only
    overwrites a transformed frame and never copies a lost frame, and every
    analysed window holds its frames in order.  Returns the states and the
    analysed batches."""
    missing = missing or [frozenset()] * len(specs)
    queue_caps = queue_caps or [1 << 30] * len(specs)
    states = [CamState(RingPlan(w, h), t, queue_cap=qc, missing=frozenset(m))
              for (w, h), t, m, qc in zip(specs, targets, missing, queue_caps)]
    sched = Scheduler(states, max_batch, per_camera)
    u16 = [np.full(s.ring.R, -1) for s in states]
    holo = [np.full(s.ring.slots, -1) for s in states]
    transformed = [set() for _ in states]
    lost = [set() for _ in states]
    batches = []
    for avail in arrivals:
        for a in sched.step(avail):
            if a[0] == "copy":
                _, i, lo, hi, lost_here = a
                lost[i] |= set(lost_here)
                for k in range(lo, hi):
                    if k in lost_here:
                        continue
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
                    assert not (set(want.tolist()) & lost[i]), f"camera {i} window {c} holds a lost frame"
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


def test_gaps_skip_and_count_windows():
    # sequence numbers 40 and 41 never arrive: window 1 (frames 25..56) is skipped,
    # every other window is analysed in order
    st, batches = _simulate([(32, 25)], [6], [[10 ** 9]] * 100, missing=[{40, 41}])
    s = st[0]
    assert s.done() and s.gaps == 2 and s.dropped == 0 and s.skipped == 1 and s.analysed == 5
    assert [c for b in batches for _, c in b] == [0, 2, 3, 4, 5]


def test_gap_in_overlap_skips_both_windows():
    # frame 27 lies in windows 0 (0..31) and 1 (25..56)
    st, batches = _simulate([(32, 25)], [4], [[10 ** 9]] * 100, missing=[{27}])
    assert st[0].skipped == 2 and [c for b in batches for _, c in b] == [2, 3]


def test_bounded_ingest_queue_drops_and_counts():
    # frames arrive 200 per pass while each pass consumes at most two windows (50
    # frames) and the ring admits at most R frames past the oldest pending window:
    # the 30-frame ingest queue overflows; every window is analysed or skipped, none
    # analysed holds a lost frame (checked in the simulation)
    n = 40
    arrivals = [[200 * t] for t in range(1, 200)]
    st, batches = _simulate([(32, 25)], [n], arrivals, per_camera=2, queue_caps=[30])
    s = st[0]
    assert s.done()
    assert s.dropped > 0 and s.gaps == 0
    assert s.analysed + s.skipped == n and s.analysed == sum(len(b) for b in batches)
    assert s.skipped > 0


def test_queue_large_enough_drops_nothing():
    arrivals = [[25 * t] for t in range(1, 400)]   # one hop per pass: the consumer keeps up
    st, batches = _simulate([(32, 25)], [20], arrivals, per_camera=2, queue_caps=[64])
    assert st[0].dropped == 0 and st[0].skipped == 0 and st[0].analysed == 20


def test_disconnect_stops_scheduling():
    states = [CamState(RingPlan(32, 25), 10), CamState(RingPlan(32, 25), 10)]
    sched = Scheduler(states)
    sched.step([100, 100])
    states[1].stopped = True
    assert states[1].done()
    before = states[1].analysed
    for _ in range(20):
        for a in sched.step([10 ** 6, 10 ** 6]):
            cams = {i for i, _ in a[1]} if a[0] == "analyse" else {a[1]}
            assert cams == {0}, f"a disconnected camera was scheduled: {a[:2]}"
    assert states[0].done() and states[1].analysed == before < 10


def test_admission_release_and_queued_request():
    # a budget for one camera at a time: B waits until A is released, then fits;
    # the named scheduler takes B in mid-run
    a = CameraSpec("A", 1024, 1024, 500.0, 100)
    b = CameraSpec("B", 1024, 2048, 250.0, 101)
    ra, rb = RingPlan(32, 25), RingPlan(32, 25)
    need_b = sum(camera_bytes(b, rb, 4).values())
    adm = Admission(need_b)
    adm.request(a, ra)
    assert not adm.fits(b, rb)
    with pytest.raises(AdmissionError):
        adm.request(b, rb)
    sched = Scheduler({}, 16, 2)
    sa = CamState(ra, 3)
    sched.add("A", sa)
    pending = [("B", b, rb)]
    order = []
    for t in range(1, 400):
        if sa.done() and "A" in sched.st:
            sched.remove("A")
            assert adm.release("A") > 0
        if pending and adm.fits(pending[0][1], pending[0][2]):
            name, spec, ring = pending.pop(0)
            adm.request(spec, ring)
            sched.add(name, CamState(ring, 2))
            order.append(("admit", name, t))
        acts = sched.step({n: 25 * t for n in sched.st})
        order += [("win", i, c) for x in acts if x[0] == "analyse" for i, c in x[1]]
        if not pending and all(s.done() for s in sched.st.values()):
            break
    wins = [o for o in order if o[0] == "win"]
    assert [(i, c) for _, i, c in wins] == [("A", 0), ("A", 1), ("A", 2), ("B", 0), ("B", 1)]
    admit_b = [o for o in order if o[0] == "admit"][0]
    assert admit_b[2] > 1 and adm.held == {"B": need_b}


def test_fourier_camera_needs_no_analysis_workspace():
    from paper_2004_00923_amd.serve import CameraSpec, camera_bytes
    P = CameraSpec("P", 64, 64, 500.0, 1)
    F = CameraSpec("F", 64, 64, 500.0, 1, hop=1, k_lo=7, k_hi=23, demod="fourier", ring_hops=64)
    assert camera_bytes(P, P.ring(), 4)["workspace"] > 0
    b = camera_bytes(F, F.ring(), 4)
    assert b["workspace"] == 0
    assert F.ring().R == 64 and F.ring().slots == 64 + 31


@pytest.mark.parametrize("window,hop,ring_hops", [(32, 1, 96), (32, 25, 6), (16, 40, 6), (3, 2, 2)])
@pytest.mark.parametrize("n_images", [1, 4, 7])
def test_window_runs_contiguous(window, hop, ring_hops, n_images):
    # the runs of ready windows rendered by one launch: they partition the ready list,
    # each run's frames lie in one stretch of the ring (position s0 + j holds frame
    # c0 hop + j, in its own slot or in a mirror copy) and its images do not wrap
    r = RingPlan(window, hop, ring_hops)
    rng = np.random.default_rng(window + hop + n_images)
    for _ in range(60):
        start = int(rng.integers(0, 500))
        cs = sorted({start + int(d) for d in rng.integers(0, 40, size=int(rng.integers(1, 30)))})
        runs = r.window_runs(cs, n_images)
        assert [c0 + j for c0, k in runs for j in range(k)] == cs
        for c0, k in runs:
            s0 = r.window_slot(c0)
            assert s0 + (k - 1) * hop + window <= r.slots
            assert c0 % n_images + k <= n_images
            for j in range((k - 1) * hop + window):
                pos, slot = s0 + j, (c0 * hop + j) % r.R
                assert pos == slot or (pos - r.R == slot and slot < r.M)
