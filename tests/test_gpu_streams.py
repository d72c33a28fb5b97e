"""Work of one context on two streams at once.

The library keeps its FFT and evaluation scratch per stream, so prefilters
and evaluations of different fields issued on two streams of the same context
(the benchmark overlaps the two halves of a step this way) must give exactly
the results of the same calls issued one after another on one stream.
"""
import numpy as np
import pytest

import synth
from gpu_common import log, dev

pytestmark = pytest.mark.gpu


def test_two_streams_match_one_stream():
    import torch
    import paper_1201_4060_amd as bsi
    n, C, P = 48, 3, 20000
    ctx = bsi.Context(0)
    fields = {}
    try:
        for N in (4, 6):
            fields[N] = bsi.Field(ctx, n, C, N, bsi.BSI_F32)
        uhat = {N: dev(synth.kolmogorov_spectrum(n, C, seed=700 + N)) for N in fields}
        pos = {N: dev(synth.uniform_positions(P, seed=710 + N)) for N in fields}

        def run(N):
            fields[N].set_spectrum(uhat[N])
            return fields[N].eval(pos[N])

        ref = {N: run(N) for N in fields}
        torch.cuda.synchronize()
        ref = {N: (u.clone(), g.clone()) for N, (u, g) in ref.items()}
        main = torch.cuda.current_stream()
        side = torch.cuda.Stream()
        for rep in range(3):
            side.wait_stream(main)
            with torch.cuda.stream(side):
                got6 = run(6)
            got4 = run(4)
            main.wait_stream(side)
            torch.cuda.synchronize()
            for N, (u, g) in ((4, got4), (6, got6)):
                assert torch.equal(u, ref[N][0]) and torch.equal(g, ref[N][1]), f"rep {rep} order {N}"
            log(f"  rep {rep}: both orders bitwise equal to the one-stream results")
    finally:
        for f in fields.values():
            f.close()
        ctx.close()
