"""Boundary behaviour of the C ABI on the GPU: queue-full backpressure (PW_EBUSY), error
messages written from two threads at once, device inputs that need a cast or a copy first, and
host inputs in pageable and in pinned memory (staged through the context's pinned pool).

Two runs of one request agree to FP64 rounding, not bit for bit: the shell sums are FP64
partial sums combined across workgroups in the order they finish; the painted mesh and the
bin counts are exact."""
import threading

import numpy as np
import pytest

from synthetic import WORKLOADS, make_workload_catalog, to_xyzw

from gpu_common import say, uniform_catalog, max_err_per_ell

pytestmark = pytest.mark.gpu

pw = pytest.importorskip("paper_2102_08384_amd.pw")
torch = pytest.importorskip("torch")


SAME = 1e-12   # two runs of one request, in units of the monopole scale


def _small_cfg(**kw):
    base = dict(stat=pw.PW_PK, los=pw.PW_BISECTOR, assign=pw.PW_TSC, prec=pw.PW_FP32, n_mesh=64,
                box_len=1000.0, box_origin=(-500.0, -500.0, 600.0), ell_max=4, order=4, compensate=1,
                bin_lo=0.005, bin_width=0.02, n_bins=9)
    base.update(kw)
    return pw.Config(**base)


def test_queue_limit_refuses_with_ebusy():
    """One lane and a limit of two requests in flight: a third submission, made while the
    first (a 512^3 estimate on a fresh context) cannot have finished, is refused with PW_EBUSY
    and enqueues nothing; once the two complete, submissions are accepted again."""
    say("queue limit: 2 in flight on one lane, third submission refused")
    gal, ran = make_workload_catalog("C3", index=0, n_gal=500_000)
    wl = WORKLOADS["C3"]
    gx = torch.from_numpy(to_xyzw(gal, np.float32)).cuda()
    rx = torch.from_numpy(to_xyzw(ran, np.float32)).cuda()
    rn = torch.from_numpy(ran["nbar"].astype(np.float32)).cuda()
    cfg = pw.Config(stat=pw.PW_PK, los=pw.PW_BISECTOR, assign=pw.PW_TSC, prec=pw.PW_FP32, n_mesh=512,
                    box_len=wl.L, box_origin=wl.b0, ell_max=4, order=4, compensate=1, bin_lo=0.005,
                    bin_width=0.005, n_bins=79)
    with pw.Context(0) as ctx:
        ctx.set_lanes(1)
        ctx.set_queue_limit(2)
        a = ctx.submit(cfg, gx, rx, ran_nbar=rn)
        b = ctx.submit(cfg, gx, rx, ran_nbar=rn)
        with pytest.raises(pw.PwError) as ei:
            ctx.submit(cfg, gx, rx, ran_nbar=rn)
        assert ei.value.code == pw.PW_EBUSY
        assert "queue is full" in ctx.last_error()
        ra, rb = a.wait(), b.wait()
        assert np.all(max_err_per_ell(rb["values"], ra["values"]) < SAME)
        d = ctx.submit(cfg, gx, rx, ran_nbar=rn).wait()
        assert np.all(max_err_per_ell(d["values"], ra["values"]) < SAME)
        with pytest.raises(pw.PwError) as ei:
            ctx.set_queue_limit(0)
        assert ei.value.code == pw.PW_EINVAL


def test_error_messages_from_two_threads():
    """pw_estimate failing on one thread while pw_submit / pw_poll fail on another: each call
    returns its own code and pw_last_error always reads one whole message."""
    say("last error: two threads failing at once")
    gal, ran = uniform_catalog(7, 200, 600, (0, 0, 1000), 300)
    gx, rx = to_xyzw(gal, np.float32), to_xyzw(ran, np.float32)
    nb = ran["nbar"].astype(np.float32)
    bad_mesh = _small_cfg(n_mesh=48)        # not a power of two
    bad_ell = _small_cfg(ell_max=3)         # odd multipole
    with pw.Context(0) as ctx:
        msgs = {}
        for name, cfg in (("mesh", bad_mesh), ("ell", bad_ell)):
            with pytest.raises(pw.PwError):
                ctx.estimate(cfg, gx, rx, ran_nbar=nb)
            msgs[name] = ctx.last_error()
        assert msgs["mesh"] and msgs["ell"] and msgs["mesh"] != msgs["ell"]
        allowed = set(msgs.values()) | {"", "cancelled"}
        seen, errors = [], []

        def estimating():
            for _ in range(400):
                try:
                    ctx.estimate(bad_mesh, gx, rx, ran_nbar=nb)
                    errors.append("estimate did not fail")
                except pw.PwError as e:
                    if e.code != pw.PW_EINVAL:
                        errors.append(str(e))
                seen.append(ctx.last_error())

        def submitting():
            for _ in range(400):
                try:
                    ctx.submit(bad_ell, gx, rx, ran_nbar=nb)
                    errors.append("submit did not fail")
                except pw.PwError as e:
                    if e.code != pw.PW_EINVAL:
                        errors.append(str(e))
                seen.append(ctx.last_error())

        ts = [threading.Thread(target=estimating), threading.Thread(target=submitting)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        assert not errors, errors[:3]
        assert len(seen) == 800 and set(seen) <= allowed, set(seen) - allowed


def test_device_inputs_after_cast_and_copy():
    """Device tensors that the binding must cast (an FP64 nbar beside FP32 positions) or copy (a
    non-contiguous view) give the same result as prepared FP32 inputs."""
    say("device inputs: cast nbar, non-contiguous positions")
    gal, ran = uniform_catalog(11, 20000, 60000, (0, 0, 1000), 400)
    cfg = _small_cfg()
    gx = torch.from_numpy(to_xyzw(gal, np.float32)).cuda()
    rx = torch.from_numpy(to_xyzw(ran, np.float32)).cuda()
    rn32 = torch.from_numpy(ran["nbar"].astype(np.float32)).cuda()
    rn64 = torch.from_numpy(ran["nbar"].astype(np.float32).astype(np.float64)).cuda()
    wide = torch.zeros((rx.shape[0], 8), dtype=torch.float32, device="cuda")
    wide[:, 2:6] = rx
    view = wide[:, 2:6]
    assert not view.is_contiguous()
    with pw.Context(0) as ctx:
        ref = ctx.estimate(cfg, gx, rx, ran_nbar=rn32)
        got = ctx.estimate(cfg, gx, view, ran_nbar=rn64)
        sub = ctx.submit(cfg, gx, view, ran_nbar=rn64).wait()
    assert np.all(max_err_per_ell(got["values"], ref["values"]) < SAME)
    assert np.all(max_err_per_ell(sub["values"], ref["values"]) < SAME)
    assert np.allclose(got["norm"], ref["norm"], rtol=1e-14, atol=0)


def test_host_inputs_pageable_and_pinned():
    """The same request from device memory, from pageable host memory (copied into the
    context's pinned pool at submission) and from pinned host memory (read in place), several
    in flight together on two lanes: every result is the device-input result."""
    say("host inputs: pageable and pinned, served together")
    gal, ran = uniform_catalog(13, 30000, 90000, (0, 0, 1000), 420)
    cfg = _small_cfg(n_mesh=128)
    gx, rx = to_xyzw(gal, np.float32), to_xyzw(ran, np.float32)
    nb = ran["nbar"].astype(np.float32)
    dev = [torch.from_numpy(a).cuda() for a in (gx, rx, nb)]
    pinned = [torch.from_numpy(a).pin_memory() for a in (gx, rx, nb)]
    assert pinned[0].is_pinned()
    with pw.Context(0) as ctx:
        ctx.set_lanes(2)
        ref = ctx.estimate(cfg, *dev[:2], ran_nbar=dev[2])
        plain_host = ctx.estimate(cfg, gx, rx, ran_nbar=nb)
        tickets = []
        for _ in range(3):
            tickets.append(ctx.submit(cfg, gx, rx, ran_nbar=nb))
            tickets.append(ctx.submit(cfg, *pinned[:2], ran_nbar=pinned[2]))
            tickets.append(ctx.submit(cfg, *dev[:2], ran_nbar=dev[2]))
        res = [t.wait() for t in tickets]
    assert np.all(max_err_per_ell(plain_host["values"], ref["values"]) < SAME)
    for r in res:
        assert np.all(max_err_per_ell(r["values"], ref["values"]) < SAME)
        assert np.array_equal(r["counts"], ref["counts"])
