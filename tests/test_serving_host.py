"""Serving admission rule and arena allocator, exercised on the host through
xs_sched_simulate (the same policy and allocator the server thread uses), against
independent checks: a plain FIFO multi-server queue, capacity invariants over time, the
bypass bound, and the arena's exact rounding."""
import numpy as np
import pytest

from paper_2510_20870_amd import xsec

pytestmark = pytest.mark.skipif(not __import__("os").path.exists(xsec.LIB_PATH),
                                reason="libxsec.so not built")


def r256(b):
    return (np.maximum(np.asarray(b, np.uint64), 1) + 255) // 256 * 256


def fifo_reference(arrive, dur, slots):
    """Plain FIFO queue with `slots` identical servers (memory never binds)."""
    free_at = [0.0] * slots
    admit = np.zeros(len(arrive))
    for i, (a, d) in enumerate(zip(arrive, dur)):
        k = int(np.argmin(free_at))
        admit[i] = max(a, free_at[k])
        free_at[k] = admit[i] + d
    return admit


def check_capacity(admit, done, fp, mem, slots):
    """At every admission instant the running set fits the slots and the arena."""
    for t in np.unique(admit):
        run = (admit <= t) & (done > t)
        assert run.sum() <= slots
        assert int(r256(fp[run]).sum()) <= mem


def test_fifo_when_memory_never_binds():
    rng = np.random.default_rng(0)
    n = 300
    arrive = np.cumsum(rng.exponential(1.0, n))
    dur = rng.uniform(0.5, 6.0, n)
    fp = rng.integers(1, 1000, n).astype(np.uint64)
    for slots in (1, 2, 4, 7):
        admit, done, peak = xsec.sched_simulate(arrive, dur, fp, 1 << 30, slots)
        np.testing.assert_allclose(admit, fifo_reference(arrive, dur, slots), rtol=0, atol=0)
        np.testing.assert_allclose(done, admit + dur, rtol=0, atol=0)
        assert peak <= int(r256(fp).sum())


def test_capacity_invariants_random_mix():
    rng = np.random.default_rng(1)
    n = 400
    arrive = np.cumsum(rng.exponential(0.3, n))
    dur = rng.uniform(0.1, 3.0, n)
    mem = 1 << 20
    fp = rng.integers(1, mem // 3, n).astype(np.uint64)
    for slots, bypass in ((4, 8), (2, 1), (8, -1), (3, 1000)):
        admit, done, peak = xsec.sched_simulate(arrive, dur, fp, mem, slots, bypass)
        assert np.all(admit >= arrive)
        np.testing.assert_allclose(done, admit + dur, rtol=0, atol=0)
        check_capacity(admit, done, fp, mem, slots)
        assert peak <= mem


def test_strict_fifo_order_without_bypass():
    rng = np.random.default_rng(2)
    n = 200
    arrive = np.cumsum(rng.exponential(0.2, n))
    dur = rng.uniform(0.1, 2.0, n)
    mem = 1 << 16
    fp = rng.integers(1, mem, n).astype(np.uint64)
    admit, done, _ = xsec.sched_simulate(arrive, dur, fp, mem, 4, -1)
    assert np.all(np.diff(admit) >= 0), "max_bypass < 0 must admit in arrival order"
    check_capacity(admit, done, fp, mem, 4)


def test_small_requests_pass_a_blocked_large_one_a_bounded_number_of_times():
    mem = 1 << 20
    # request 0 holds 3/4 of the arena for a long time; request 1 needs 1/2 and waits;
    # requests 2.. need 1/16 each and arrive behind it
    arrive = np.array([0.0, 0.1] + [0.2 + 0.01 * k for k in range(10)])
    dur = np.array([10.0, 1.0] + [0.5] * 10)
    fp = np.array([3 * mem // 4, mem // 2] + [mem // 16] * 10, np.uint64)
    for bypass in (1, 3, 5):
        admit, done, _ = xsec.sched_simulate(arrive, dur, fp, mem, 16, bypass)
        passed = int(np.sum(admit[2:] < admit[1]))
        assert passed == bypass, (bypass, admit)
        assert admit[1] == pytest.approx(10.0, abs=0)   # admitted as soon as 0 is done
        check_capacity(admit, done, fp, mem, 16)
    admit, _, _ = xsec.sched_simulate(arrive, dur, fp, mem, 16, -1)
    assert np.all(admit[2:] >= admit[1])


def test_arena_rounding_and_reuse():
    # 256-byte units: 1 byte takes 256, 257 takes 512
    admit, done, peak = xsec.sched_simulate([0, 0, 0], [1, 1, 1], [1, 257, 256], 1024, 3)
    assert peak == 256 + 512 + 256
    assert np.all(admit == 0)
    # an arena of exactly four units fits four one-unit requests, the fifth waits
    admit, _, peak = xsec.sched_simulate([0] * 5, [1] * 5, [200] * 5, 1024, 8)
    assert list(admit) == [0, 0, 0, 0, 1] and peak == 1024


def test_fragmentation_is_merged_on_release():
    # A B C D fill the arena; B and C finish, then a request of B+C's size must fit in the
    # merged hole while A and D still run
    u = 256
    arrive = [0, 0, 0, 0, 0.5]
    dur = [10, 1, 1, 10, 1]
    fp = [u, u, u, u, 2 * u]
    admit, _, _ = xsec.sched_simulate(arrive, dur, fp, 4 * u, 8)
    assert admit[4] == 1.0


def test_oversized_and_invalid_requests_are_rejected():
    with pytest.raises(xsec.XsError) as e:
        xsec.sched_simulate([0], [1], [2048], 1024, 1)
    assert e.value.code == xsec.XS_ENOMEM
    with pytest.raises(xsec.XsError) as e:
        xsec.sched_simulate([1, 0], [1, 1], [1, 1], 1024, 1)
    assert e.value.code == xsec.XS_EINVAL
    with pytest.raises(xsec.XsError):
        xsec.sched_simulate([0], [1], [1], 1024, 0)
    a, d, p = xsec.sched_simulate([], [], [], 1024, 1)
    assert len(a) == 0 and p == 0
