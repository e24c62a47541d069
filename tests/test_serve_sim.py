"""Serving scheduler on the CPU: the engine driven step by step with the
simulated executor (modelled time, no device work).  Checks admission by
memory footprint and slots, first-come-first-served order, continuous
batching, rejection and back-pressure, and that memory and slots return."""

import numpy as np
import pytest

from paper_2409_07413_amd import binding as B


def sched():
    # 3 blocks: (HIO^j ER^(7-j)), SW; final GetError
    return B.sched_plain(alg=B.ALG_HIO, G=3, j=4, j_er=3, j_end=0, beta=0.9, chi=0.5, sigma=2.0,
                         sigma_end=1.0, tau=0.1, tau_end=0.1)


def server(budget=64 << 20, max_shots=8, P=4, launch_s=5e-6, **kw):
    return B.Server(None, sched(), P=P, hbm_budget=budget, max_shots=max_shots, manual=True,
                    sim_bytes_per_s=1e12, sim_launch_s=launch_s, **kw)


def shot(n):
    return (np.ones((n, n), np.float32), np.ones((n, n), np.uint8), np.ones((n, n), np.uint8))


def run(sv):
    steps = 0
    while sv.step():
        steps += 1
        assert steps < 100000
    return steps


def footprint(n, P=4):
    sv = server(P=P)
    t = sv.submit(*shot(n), arrival=0.0)
    sv.step()
    fp = sv.stats()["bytes_in_use"]
    run(sv)
    sv.poll(t, want_data=False)
    sv.close()
    return fp


def test_single_shot_runs_one_tick_per_sequence():
    sv = server()
    t = sv.submit(*shot(32), arrival=0.0)
    run(sv)
    r = sv.poll(t, want_data=False)
    st = sv.stats()
    assert st["ticks"] == 3  # one per sequence; SW and GetError ride on the ticks
    assert st["admitted"] == st["completed"] == 1
    assert st["bytes_in_use"] == 0 and st["bytes_peak"] > 0
    assert 0.0 == r["t_arrival"] == r["t_admit"] < r["t_finish"]
    with pytest.raises(B.SprError):
        sv.poll(t)  # the ticket is forgotten once read
    sv.close()


def test_footprint_grows_with_size_and_members():
    assert footprint(64) > footprint(32)
    assert footprint(32, P=8) > footprint(32, P=4)
    # densities and row transforms dominate: about 16 bytes per member pixel
    fp = footprint(128, P=4)
    assert 16 * 4 * 128 * 128 <= fp <= 24 * 4 * 128 * 128


def test_admission_by_memory_footprint():
    fp = footprint(64)
    # budget for exactly two shots of 64^2 (plus less than a third)
    sv = server(budget=int(2.5 * fp), max_shots=16)
    ts = [sv.submit(*shot(64), arrival=0.0) for _ in range(5)]
    sv.step()
    st = sv.stats()
    assert st["active"] == 2 and st["queued"] == 3
    run(sv)
    res = [sv.poll(t, want_data=False) for t in ts]
    st = sv.stats()
    assert st["max_active"] == 2
    assert st["bytes_peak"] <= st["bytes_capacity"]
    assert st["bytes_in_use"] == 0 and st["completed"] == 5
    # first come, first served
    admits = [r["t_admit"] for r in res]
    assert admits == sorted(admits)
    # the third shot waits for the first two to finish
    assert res[2]["t_admit"] >= min(res[0]["t_finish"], res[1]["t_finish"])
    sv.close()


def test_slot_limit():
    sv = server(max_shots=3)
    ts = [sv.submit(*shot(32), arrival=0.0) for _ in range(7)]
    run(sv)
    assert sv.stats()["max_active"] == 3
    for t in ts:
        assert sv.poll(t, want_data=False) is not None
    sv.close()


def test_continuous_batching_admits_while_others_run():
    sv = server()
    a = sv.submit(*shot(64), arrival=0.0)
    # arrives during a's first tick: joins at the next tick, before a finishes
    b = sv.submit(*shot(64), arrival=1e-9)
    run(sv)
    ra, rb = sv.poll(a, want_data=False), sv.poll(b, want_data=False)
    assert rb["t_admit"] < ra["t_finish"]
    assert rb["t_admit"] > ra["t_admit"]
    sv.close()


def test_same_size_shots_share_launches():
    def launches(k):
        sv = server()
        ts = [sv.submit(*shot(32), arrival=0.0) for _ in range(k)]
        run(sv)
        for t in ts:
            sv.poll(t, want_data=False)
        n = sv.stats()["launches"]
        sv.close()
        return n

    one, four = launches(1), launches(4)
    # uploads and result copies are per shot; iterations, SW and GetError are shared
    assert four < 2 * one


def test_mixed_sizes_and_arrivals_complete_in_order_of_service():
    rng = np.random.default_rng(4005)
    sizes = rng.choice([32, 48, 64, 96], size=30)
    arrivals = np.cumsum(rng.exponential(2e-4, size=30))
    sv = server(max_shots=4)
    ts = [sv.submit(*shot(int(n)), arrival=float(t)) for n, t in zip(sizes, arrivals)]
    run(sv)
    res = [sv.poll(t, want_data=False) for t in ts]
    for r, t in zip(res, arrivals):
        assert r["t_arrival"] == pytest.approx(t)
        assert r["t_arrival"] <= r["t_admit"] < r["t_finish"]
    admits = [r["t_admit"] for r in res]
    assert admits == sorted(admits)
    st = sv.stats()
    assert st["completed"] == 30 and st["bytes_in_use"] == 0 and st["max_active"] <= 4
    sv.close()


def test_rejections_and_back_pressure():
    fp = footprint(64)
    sv = server(budget=int(1.5 * fp), max_queue=2)
    with pytest.raises(B.SprError) as e:
        sv.submit(*shot(128), arrival=0.0)  # can never fit
    assert e.value.code == B.E_ADMISSION
    with pytest.raises(B.SprError) as e:
        sv.submit(*shot(100), arrival=0.0)  # no kernels for this size
    assert e.value.code == -2
    amp, mask, supp = shot(32)
    amp[3, 4] = -1.0
    with pytest.raises(B.SprError) as e:
        sv.submit(amp, mask, supp, arrival=0.0)
    assert e.value.code == -7
    t1 = sv.submit(*shot(64), arrival=0.0)
    t2 = sv.submit(*shot(64), arrival=0.0)
    with pytest.raises(B.SprError) as e:
        sv.submit(*shot(64), arrival=0.0)  # queue of two is full
    assert e.value.code == B.E_BUSY
    sv.step()  # t1 admitted: room in the queue again
    t3 = sv.submit(*shot(64), arrival=0.0)
    run(sv)
    for t in (t1, t2, t3):
        assert sv.poll(t, want_data=False) is not None
    sv.close()


def test_invalid_configurations():
    with pytest.raises(B.SprError):
        B.Server(None, sched(), P=4, hbm_budget=1 << 20, max_shots=2, manual=False, sim_bytes_per_s=1e12)
    with pytest.raises(B.SprError):
        B.Server(None, sched(), P=4, hbm_budget=1 << 20, max_shots=2, manual=True, sim_bytes_per_s=0.0)
    with pytest.raises(B.SprError):
        B.Server(None, sched(), P=0, hbm_budget=1 << 20, max_shots=2, manual=True, sim_bytes_per_s=1e12)
    memetic = B.sched_ops([B.op(B.OP_SELECT, gen=1)])
    with pytest.raises(B.SprError):
        B.Server(None, memetic, P=4, hbm_budget=1 << 20, max_shots=2, manual=True, sim_bytes_per_s=1e12)


def test_shortest_first_lets_small_shots_pass():
    # bandwidth-dominated model (negligible launch cost), sizes 16x apart in pixels
    def run_pair(shortest):
        sv = server(max_shots=2, shortest_first=shortest, launch_s=1e-9)
        big = sv.submit(*shot(128), arrival=0.0)
        small = sv.submit(*shot(32), arrival=1e-9)
        run(sv)
        rb, rs = sv.poll(big, want_data=False), sv.poll(small, want_data=False)
        sv.close()
        return rb, rs

    def alone(n):
        sv = server(launch_s=1e-9)
        t = sv.submit(*shot(n), arrival=0.0)
        run(sv)
        r = sv.poll(t, want_data=False)
        sv.close()
        return r["t_finish"] - r["t_arrival"]

    lat = lambda r: r["t_finish"] - r["t_arrival"]  # noqa: E731
    rb0, rs0 = run_pair(False)
    rb1, rs1 = run_pair(True)
    # lockstep: the small shot advances one sequence per tick of the big one
    assert lat(rs0) > 0.5 * alone(128)
    # shortest first: it waits for the big shot's tick in progress, then runs alone
    assert lat(rs1) <= alone(32) + alone(128) / 3 * 1.05
    assert rs1["t_finish"] < rb1["t_finish"]
    # the big shot is delayed by about the small one's work
    assert lat(rb1) <= alone(128) + alone(32) * 1.05


def test_shortest_first_does_not_starve_large_shots():
    sv = server(max_shots=2, shortest_first=True)
    big = sv.submit(*shot(96), arrival=0.0)
    svc = 3e-5  # arrivals of small shots closer than their own service time: a persistent queue
    smalls = [sv.submit(*shot(32), arrival=1e-6 + k * svc) for k in range(60)]
    run(sv)
    rb = sv.poll(big, want_data=False)
    last = max(sv.poll(t, want_data=False)["t_finish"] for t in smalls)
    assert rb["t_finish"] < last  # aging lets the large shot through before the stream of small ones ends
    sv.close()
