"""GPU: hh_analyze_batch (steps (b)-(e) on caller-held holograms) and the
streaming server built on it: sliding windows over two cameras, continuous
batching, images equal alone and mixed, and equal to the oracle."""
import numpy as np
import pytest

import oracle
from gpu_util import LAM, PITCH, Z, rel, say, to_dev, to_np
from paper_2004_00923_amd.synth import gen_stack

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-5


@pytest.fixture(scope="module")
def hh():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2004_00923_amd.hh as hh_mod
    hh_mod.lib()
    return hh_mod


def test_analyze_batch_equals_pipeline(hh):
    # holograms from hh_fresnel, analysed in one uneven batch (one a view into a
    # larger ring), must give exactly the hh_pipeline image of each stack
    import torch
    specs = [(32, 64, 64, 2), (16, 32, 128, 3), (32, 128, 128, 2)]
    ps, holos, imgs, ref, host = [], [], [], [], []
    ring = None
    for i, (nt, ny, nx, k_lo) in enumerate(specs):
        f = gen_stack(200 + i, nt, ny, nx)
        host.append(f)
        p = hh.Params(nx=nx, ny=ny, nt=nt, k_lo=k_lo, k_hi=nt - 1)
        ps.append(p)
        if i == 2:
            ring = torch.empty((nt + 9, ny, nx), dtype=torch.complex64, device="cuda")
            H = ring[5:5 + nt]
        else:
            H = torch.empty((nt, ny, nx), dtype=torch.complex64, device="cuda")
        hh.hh_fresnel(p, to_dev(f), H)
        holos.append(H)
        imgs.append(torch.empty((ny, nx), dtype=torch.float32, device="cuda"))
        ws = hh.alloc_workspace(hh.workspace_bytes(p))
        img = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
        hh.hh_pipeline(p, to_dev(f), img, ws)
        ref.append(to_np(img))
    ws = hh.alloc_workspace(hh.analyze_batch_workspace_bytes(ps))
    evs = [torch.empty(p.nt, dtype=torch.float64, device="cuda") for p in ps]
    hh.hh_analyze_batch(ps, holos, imgs, ws, evals=evs)
    for i, p in enumerate(ps):
        M = to_np(imgs[i])
        assert np.array_equal(M, ref[i]), f"stack {i}"
        r = oracle.pipeline_ref(host[i], LAM, Z, PITCH, p.k_lo, p.k_hi)
        assert rel(M, r["image"]) <= IMG_TOL
        assert np.abs(to_np(evs[i]) - r["evals"]).max() <= 1e-6 * r["evals"][0]


def test_analyze_batch_rejects_small_workspace(hh):
    import torch
    p = hh.Params(nx=32, ny=32, nt=8, k_lo=1, k_hi=7)
    H = torch.zeros((8, 32, 32), dtype=torch.complex64, device="cuda")
    img = torch.empty((32, 32), dtype=torch.float32, device="cuda")
    need = hh.analyze_batch_workspace_bytes([p])
    ws = hh.alloc_workspace(need - 256)
    with pytest.raises(hh.HHError) as ei:
        hh.hh_analyze_batch([p], [H], [img], ws)
    assert ei.value.status == hh.HH_E_WORKSPACE


def _source(seed, n, ny, nx):
    import torch
    f = gen_stack(seed, n, ny, nx)
    t = torch.empty(f.shape, dtype=torch.uint16, pin_memory=True)
    t.copy_(torch.from_numpy(f))
    return f, t


def _serve(cams, sources, windows, paced, keep):
    from paper_2004_00923_amd.serve import Server
    srv = Server(hbm_budget_bytes=8 << 30)
    for spec in cams:
        srv.admit(spec, sources[spec.name][1])
    srv.keep_windows = set(keep)
    res = srv.run(windows, paced=paced)
    return srv, res


def test_serve_two_cameras_alone_vs_mix_and_oracle(hh):
    from paper_2004_00923_amd.serve import CameraSpec, summarize
    A = CameraSpec("A", 128, 128, 500.0, 100)
    B = CameraSpec("B", 128, 256, 250.0, 101)
    n_src = 48
    src = {"A": _source(A.seed, n_src, A.ny, A.nx), "B": _source(B.seed, n_src, B.ny, B.nx)}
    wa, wb = 5, 3
    keepA = [("A", c) for c in range(wa)]
    keepB = [("B", c) for c in range(wb)]
    say("serve: camera A alone, paced")
    alone, res_a = _serve([A], src, {"A": wa}, True, keepA)
    say("serve: cameras A + B, paced")
    mix, res_m = _serve([A, B], src, {"A": wa, "B": wb}, True, keepA + keepB)
    say("serve: cameras A + B, unthrottled")
    fast, res_f = _serve([A, B], src, {"A": wa, "B": wb}, False, keepA + keepB)
    s = summarize(res_m, [A, B])
    say(f"serve summary (mixed, paced): {s}")
    assert len(res_m["windows"]) == wa + wb
    assert all(w["latency_ms"] > 0 for w in res_m["windows"])
    for c in range(wa):
        a = to_np(alone.kept[("A", c)])
        assert np.array_equal(a, to_np(mix.kept[("A", c)])), f"A window {c}: mixed differs from alone"
        assert np.array_equal(a, to_np(fast.kept[("A", c)])), f"A window {c}: unthrottled differs"
    for name, spec, nw in (("A", A, wa), ("B", B, wb)):
        frames = src[name][0]
        for c in range(nw):
            idx = [(c * spec.hop + j) % n_src for j in range(spec.window)]
            r = oracle.pipeline_ref(frames[idx], LAM, Z, PITCH, 2, 31)
            e = rel(to_np(mix.kept[(name, c)]), r["image"])
            assert e <= IMG_TOL, f"{name} window {c}: {e:.2e}"


def test_serve_admission_rejects_over_budget(hh):
    import torch
    from paper_2004_00923_amd.serve import AdmissionError, CameraSpec, RingPlan, Server, camera_bytes
    A = CameraSpec("A", 128, 128, 500.0, 100)
    B = CameraSpec("B", 128, 256, 250.0, 101)
    need_a = sum(camera_bytes(A, A.ring(), 4).values())
    srv = Server(hbm_budget_bytes=need_a + 1024)
    srv.admit(A, torch.zeros((4, 128, 128), dtype=torch.uint16, pin_memory=True))
    with pytest.raises(AdmissionError):
        srv.admit(B, torch.zeros((4, 128, 256), dtype=torch.uint16, pin_memory=True))
    assert len(srv.cams) == 1


def test_serve_alone_vs_mix_at_camera_sizes(hh):
    # camera A (1024^2, 500 frames/s) alone and mixed with camera B (2048 x 1024,
    # 250 frames/s), paced: A's images are bit-identical in both runs, and one window
    # of each camera matches the oracle at full size
    from paper_2004_00923_amd.serve import CameraSpec
    A = CameraSpec("A", 1024, 1024, 500.0, 100)
    B = CameraSpec("B", 1024, 2048, 250.0, 101)
    n_src = 57
    src = {"A": _source(A.seed, n_src, A.ny, A.nx), "B": _source(B.seed, n_src, B.ny, B.nx)}
    wa, wb = 3, 2
    keepA = [("A", c) for c in range(wa)]
    keepB = [("B", c) for c in range(wb)]
    say("serve 1024^2 alone, paced")
    alone, _ = _serve([A], src, {"A": wa}, True, keepA)
    say("serve 1024^2 + 2048x1024, paced")
    mix, res = _serve([A, B], src, {"A": wa, "B": wb}, True, keepA + keepB)
    assert len(res["windows"]) == wa + wb
    for c in range(wa):
        assert np.array_equal(to_np(alone.kept[("A", c)]), to_np(mix.kept[("A", c)])), f"A window {c}"
    for name, spec, c in (("A", A, 1), ("B", B, 1)):
        frames = src[name][0]
        idx = [(c * spec.hop + j) % n_src for j in range(spec.window)]
        r = oracle.pipeline_ref(frames[idx], LAM, Z, PITCH, 2, 31)
        e = rel(to_np(mix.kept[(name, c)]), r["image"])
        say(f"  {name} window {c} vs oracle: {e:.2e}")
        assert e <= IMG_TOL


def test_serve_queued_camera_admitted_when_memory_frees(hh):
    # the budget holds one camera: B is requested with A but waits until A has
    # produced its windows and released its memory, then joins; both are correct
    from paper_2004_00923_amd.serve import CameraRequest, CameraSpec, RingPlan, Server, camera_bytes
    A = CameraSpec("A", 128, 128, 500.0, 100)
    B = CameraSpec("B", 128, 256, 500.0, 101)
    n_src = 48
    src = {"A": _source(A.seed, n_src, A.ny, A.nx), "B": _source(B.seed, n_src, B.ny, B.nx)}
    need_b = sum(camera_bytes(B, B.ring(), 4).values())
    srv = Server(hbm_budget_bytes=need_b + 1024)
    srv.submit(CameraRequest(A, src["A"][1], windows=3))
    srv.submit(CameraRequest(B, src["B"][1], windows=2, at_s=0.01))
    srv.keep_windows = {("A", c) for c in range(3)} | {("B", c) for c in range(2)}
    res = srv.run(paced=True)
    say(f"queued admission: waits {res['admission_wait_s']} cameras {res['cameras']}")
    assert res["cameras"]["A"]["analysed"] == 3 and res["cameras"]["B"]["analysed"] == 2
    assert res["cameras"]["B"]["admitted_s"] >= res["cameras"]["A"]["released_s"]
    assert res["admission_wait_s"]["B"] > 0
    assert srv.adm.used == 0 and not srv.cams
    for name, spec, nw in (("A", A, 3), ("B", B, 2)):
        frames = src[name][0]
        for c in range(nw):
            idx = [(c * spec.hop + j) % n_src for j in range(spec.window)]
            r = oracle.pipeline_ref(frames[idx], LAM, Z, PITCH, 2, 31)
            assert rel(to_np(srv.kept[(name, c)]), r["image"]) <= IMG_TOL, f"{name} window {c}"


def test_serve_gaps_and_disconnect(hh):
    # camera A skips sequence numbers 30 and 31 (windows 0 and 1 hold them); camera B
    # disconnects early: its remaining windows are abandoned and its memory released
    from paper_2004_00923_amd.serve import CameraRequest, CameraSpec, Server
    A = CameraSpec("A", 128, 128, 500.0, 100)
    B = CameraSpec("B", 128, 128, 500.0, 102)
    n_src = 48
    src = {"A": _source(A.seed, n_src, A.ny, A.nx), "B": _source(B.seed, n_src, B.ny, B.nx)}
    srv = Server(hbm_budget_bytes=8 << 30)
    srv.submit(CameraRequest(A, src["A"][1], windows=5, missing=frozenset({30, 31})))
    srv.submit(CameraRequest(B, src["B"][1], windows=50, disconnect_s=0.15))
    srv.keep_windows = {("A", c) for c in range(5)}
    res = srv.run(paced=True)
    ca, cb = res["cameras"]["A"], res["cameras"]["B"]
    say(f"gaps/disconnect: A {ca} B {cb}")
    assert ca["gap_frames"] == 2 and ca["skipped"] == 2 and ca["analysed"] == 3
    assert set(c for n, c in srv.kept if n == "A") == {2, 3, 4}
    assert cb["abandoned"] > 0 and cb["analysed"] + cb["abandoned"] + cb["skipped"] <= 50
    assert srv.adm.used == 0
    frames = src["A"][0]
    for c in (2, 3, 4):
        idx = [(c * A.hop + j) % n_src for j in range(A.window)]
        r = oracle.pipeline_ref(frames[idx], LAM, Z, PITCH, 2, 31)
        assert rel(to_np(srv.kept[("A", c)]), r["image"]) <= IMG_TOL


def test_serve_fourier_hop1_vs_oracle_and_mixed(hh):
    # the Table 1 FFT row as a stream: a 32-frame window every frame (hop 1),
    # Eqs. (8)-(9) with the paper's band n1..n2 = 8..24 (0-based 7..23); each image
    # against the oracle's Fourier image of that window, and equal alone and beside
    # a PCA camera
    from paper_2004_00923_amd.serve import CameraSpec
    F = CameraSpec("F", 64, 128, 500.0, 120, hop=1, k_lo=7, k_hi=23, demod="fourier", ring_hops=48)
    A = CameraSpec("A", 128, 128, 500.0, 100)
    n_src = 48
    src = {"F": _source(F.seed, n_src, F.ny, F.nx), "A": _source(A.seed, n_src, A.ny, A.nx)}
    wf, wa = 12, 3
    keepF = [("F", c) for c in range(wf)]
    say("serve: Fourier camera alone, hop 1, unthrottled")
    alone, res_a = _serve([F], src, {"F": wf}, False, keepF)
    say("serve: Fourier camera beside a PCA camera, paced")
    mix, res_m = _serve([F, A], src, {"F": wf, "A": wa}, True, keepF + [("A", c) for c in range(wa)])
    assert res_a["cameras"]["F"]["analysed"] == wf and res_m["cameras"]["A"]["analysed"] == wa
    frames = src["F"][0]
    for c in range(wf):
        a = to_np(alone.kept[("F", c)])
        assert np.array_equal(a, to_np(mix.kept[("F", c)])), f"F window {c}: mixed differs from alone"
        idx = [(c + j) % n_src for j in range(F.window)]
        r = oracle.fourier_render_ref(oracle.fresnel_ref(frames[idx], LAM, Z, PITCH), 7, 23)
        e = rel(a, r)
        assert e <= IMG_TOL, f"F window {c}: {e:.2e}"
    frames_a = src["A"][0]
    for c in range(wa):
        idx = [(c * A.hop + j) % n_src for j in range(A.window)]
        r = oracle.pipeline_ref(frames_a[idx], LAM, Z, PITCH, 2, 31)
        assert rel(to_np(mix.kept[("A", c)]), r["image"]) <= IMG_TOL, f"A window {c}"
