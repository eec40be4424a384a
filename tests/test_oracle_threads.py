"""The reference's parallel loops (OpenMP over rows and tile rows) give the single-thread result bit
for bit: every output element is computed by one thread in the same order."""
import numpy as np

import afr_scenes as S


def test_thread_count_does_not_change_any_output(oracle):
    wl = S.make_workload("c1")
    cw = S.make_crosshair_workload()
    out = {}
    n_all = max(oracle.num_threads(), 4)
    try:
        for nt in (1, n_all):
            oracle.set_num_threads(nt)
            for prec in ("fp32", "fp16"):
                b, d = oracle.build_buffer(wl.stream, wl.width, wl.height, wl.k, prec, wl.t_ref)
                p = oracle.Params(t_now=wl.t_now, radius=3)
                rgb, aux, st = oracle.forward(b, p)
                planes = [getattr(b, f) for f in ("ox", "oy", "ta", "r", "g", "b", "count", "src")]
                out[nt, prec] = planes + [d, st, rgb, aux]
            xb, _ = oracle.crosshair_buffer(cw.workload.stream, cw.crosshairs, cw.workload.width,
                                            cw.workload.height, 4, cw.workload.t_ref)
            cb, _ = oracle.build_buffer(cw.workload.stream, cw.workload.width, cw.workload.height,
                                        cw.workload.k, "fp32", cw.workload.t_ref)
            out[nt, "xh"] = [oracle.estimate_crosshair(cb, xb, oracle.Params(t_now=cw.workload.t_now))]
    finally:
        oracle.set_num_threads(n_all)
    for key in ("fp32", "fp16", "xh"):
        for a, b in zip(out[1, key], out[n_all, key]):
            assert np.array_equal(np.asarray(a), np.asarray(b), equal_nan=True)
