"""Run one workload of the library from the command line and print one JSON line.

  python -m paper_1110_4623_amd.run barrier --kind xcd --nwg 2048 --lanes 256 --rounds 10000
  python -m paper_1110_4623_amd.run mutex --kind ticket --nwg 2048 --locks 1 --words 16
  python -m paper_1110_4623_amd.run sem --kind sleep --K 32 --nwg 2048
  python -m paper_1110_4623_amd.run serve --rate 1e5 --n 200000
  python -m paper_1110_4623_amd.run copy --bytes 1073741824
  python -m paper_1110_4623_amd.run micro --op ld --T 1048576 --stride 128 --ops 16

Meant for profilers (one workload per process) and quick checks.  The package decides
at import whether to use PyTorch's HIP runtime: run with SP_NO_TORCH=1 in the environment
(as bench.py does for itself) to use the system ROCm runtime instead.  `--repeat` runs
the workload that many times.
"""

from __future__ import annotations

import argparse
import json
import sys


def main(argv=None) -> int:
    from . import api

    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("what", choices=["barrier", "mutex", "sem", "serve", "copy", "micro"])
    ap.add_argument("--op", default="ld")
    ap.add_argument("--T", type=int, default=1 << 20)
    ap.add_argument("--stride", type=int, default=128)
    ap.add_argument("--mode", default="per_lane")
    ap.add_argument("--ops", type=int, default=16)
    ap.add_argument("--kind", default=None)
    ap.add_argument("--nwg", type=int, default=2048)
    ap.add_argument("--lanes", type=int, default=256)
    ap.add_argument("--rounds", type=int, default=10_000)
    ap.add_argument("--locks", type=int, default=1)
    ap.add_argument("--words", type=int, default=16)
    ap.add_argument("--total", type=int, default=1 << 20)
    ap.add_argument("--delay", type=int, default=1000)
    ap.add_argument("--K", type=int, default=32)
    ap.add_argument("--hold", type=int, default=2000)
    ap.add_argument("--rate", type=float, default=1e5)
    ap.add_argument("--n", type=int, default=200_000)
    ap.add_argument("--bytes", type=int, default=1 << 30)
    ap.add_argument("--seed", type=int, default=42)
    ap.add_argument("--repeat", type=int, default=1)
    ap.add_argument("--data", action="store_true",
                    help="sem: holders also update the guarded data (K <= 4096)")
    a = ap.parse_args(argv)
    ctx = api.Context(0)
    out = {"what": a.what}
    for _ in range(a.repeat):
        if a.what == "barrier":
            b = api.Barrier(ctx, a.kind or "xcd", a.nwg)
            try:
                _, st = b.run_hash(a.lanes, a.rounds, a.seed)
                # info() names the kind that ran (a default barrier's resolved kind)
                out.update(nwg=a.nwg, lanes=a.lanes, rounds=a.rounds,
                           us_per_round=st["kernel_ms"] * 1e3 / a.rounds, **b.info())
            finally:
                b.close()
        elif a.what == "mutex":
            m = api.Mutex(ctx, a.kind or "ticket", a.locks, a.words)
            try:
                words, st, _ = m.run(a.nwg, a.lanes, a.total, a.delay, a.seed)
                out.update(kind=a.kind or "ticket", nwg=a.nwg, total=a.total,
                           acq_per_s=a.total / (st["kernel_ms"] * 1e-3),
                           sum_words=int(words[:, 0].sum()))
            finally:
                m.close()
        elif a.what == "sem":
            s = api.Semaphore(ctx, a.kind or "sleep", a.K)
            try:
                r = s.run(a.nwg, a.lanes, a.total, a.hold, a.seed, track=False, data=a.data)
                out.update(kind=a.kind or "sleep", K=a.K, nwg=a.nwg, total=a.total,
                           pairs_per_s=a.total / (r["stats"]["kernel_ms"] * 1e-3),
                           admissions=r["state"][3])
                if a.data:
                    out["data_sum"] = int(r["data"].astype("u8").sum())
            finally:
                s.close()
        elif a.what == "serve":
            import sp_inputs
            reqs = sp_inputs.request_table(a.n, a.rate, a.seed)
            fn = api.serve if (a.kind or "persistent") == "persistent" else \
                api.serve_launch_per_request
            kw = {"nwg": min(a.nwg, 1024)} if fn is api.serve else {"streams": 4}
            _, _, res = fn(ctx, reqs, seed=a.seed, **kw)
            out.update(kind=a.kind or "persistent", rate=a.rate, n=a.n, **res)
        elif a.what == "micro":
            # a known number of agent-scope 4-byte accesses (one per lane per operation):
            # calibrates what the HBM byte counters read per such access
            import sp_inputs
            perm = sp_inputs.permutation(a.T, a.seed)
            finals, total, st = api.bench_atomic(ctx, a.op, a.nwg, a.lanes, a.T, a.stride,
                                                 a.mode, a.ops, a.seed, perm)
            out.update(op=a.op, nwg=a.nwg, lanes=a.lanes, T=a.T, stride=a.stride, mode=a.mode,
                       ops=a.ops, accesses=int(st["ops"]), ms=st["kernel_ms"])
        else:
            src, dst = ctx.zeros(a.bytes // 4), ctx.zeros(a.bytes // 4)
            st = api.copy(ctx, dst, src, a.bytes, reps=3)
            out.update(bytes=a.bytes, launches=3,
                       GB_per_s=2 * a.bytes * 3 / (st["kernel_ms"] * 1e-3) / 1e9)
        print(json.dumps(out), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
