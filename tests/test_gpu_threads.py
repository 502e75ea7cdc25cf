"""Distinct operators used from two host threads at once, each on its own stream (default
priority): every apply equals the sequential one bit for bit, and an error in one thread is that
thread's (the last-error message is per thread).  Calls on one operator must not overlap; calls on
different operators may."""
import sys
import threading

import numpy as np
import pytest

from paper_2401_12501_amd.inputs import ellipsoid_problem, sphere_problem, random_density

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_two_threads_distinct_operators():
    import torch
    from paper_2401_12501_amd import pmx
    ctx = pmx.Context(0)
    cases = []
    for k, p in enumerate((ellipsoid_problem(k=4, q=8), sphere_problem(k=4, q=8))):
        surf = pmx.Surface.from_inputs(ctx, p.surface)
        op = pmx.Operator(surf, p.a, p.grad_a)
        sig = torch.tensor(np.ascontiguousarray(random_density(p.n, 2, seed=40 + k).T), device="cuda:0")
        refs = {prec: op.apply(sig, prec).cpu().numpy() for prec in (pmx.PMX_PREC_MIXED_FMM, pmx.PMX_PREC_FP64_DIRECT)}
        cases.append((surf, op, sig, refs))
    torch.cuda.synchronize()
    mismatches, messages, failures = [], [], []

    def worker(idx, make_bad_call):
        surf, op, sig, refs = cases[idx]
        st = torch.cuda.Stream()
        try:
            st.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(st):
                for it in range(6):
                    for prec, ref in refs.items():
                        y = op.apply(sig, prec).cpu().numpy()
                        if not np.array_equal(y, ref):
                            mismatches.append((idx, it, prec))
                    if make_bad_call and it == 2:
                        try:
                            op.apply(sig, 7)
                        except pmx.PmxError as e:
                            messages.append((idx, e.code, str(e)))
            st.synchronize()
        except Exception as e:          # reported below; the other thread keeps running
            failures.append((idx, repr(e)))

    threads = [threading.Thread(target=worker, args=(0, True)), threading.Thread(target=worker, args=(1, False))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    assert not failures, failures
    assert not mismatches, mismatches
    assert len(messages) == 1 and messages[0][0] == 0 and messages[0][1] == pmx.PMX_ERR_INVALID
    assert "precision" in messages[0][2]
    say(f"[threads] two operators ({cases[0][1].N} and {cases[1][1].N} nodes) applied from two threads: "
        f"{2 * 6 * 2} applies identical to the sequential ones; the bad call's error stayed in its thread")
