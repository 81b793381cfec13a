"""Plans compiled from several host threads at once (plan compilation is
host-only): every thread gets the same kernels for the same composition, and
the error message of a failed call is the calling thread's own (thread-local
error state), while other threads keep failing and succeeding around it."""
import threading

import paper_1510_06585_amd as sk

PIPE_NSBM = [("noise", {"seed": 0x1510}), ("solarise", {}), ("blur5", {}), ("mirror", {})]


def _protos(H, W):
    return [sk.proto([H, W, 4], sk.U8)] * 2 + [sk.proto([4, 256], sk.U32), sk.proto([4], sk.U64)]


def test_concurrent_plan_compilation_and_thread_local_errors():
    ref = sk.Plan(sk.image_chain(PIPE_NSBM, "hist_sum"), _protos(777, 1234)).describe()
    errors = []

    def work(tid):
        try:
            for i in range(40):
                d = sk.Plan(sk.image_chain(PIPE_NSBM, "hist_sum"), _protos(777, 1234)).describe()
                assert d["kernels"] == ref["kernels"], "different plan"
                # a failing compile: its message names this thread's bad shape
                bad = [sk.proto([5 + tid, 7, 4], sk.U8), sk.proto([6 + tid, 7, 4], sk.U8)]
                try:
                    sk.Plan(sk.image_chain(PIPE_NSBM), bad)
                    raise AssertionError("mismatched shapes accepted")
                except sk.SkelError as e:
                    assert e.status == sk.ESHAPE
                    assert f"{6 + tid}" in str(e) and f"{5 + tid}" in str(e), str(e)
        except BaseException as e:   # noqa: BLE001 - reported by the main thread
            errors.append((tid, repr(e)))

    ts = [threading.Thread(target=work, args=(t,)) for t in range(8)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errors, errors
