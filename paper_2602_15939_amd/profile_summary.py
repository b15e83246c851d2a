"""Summarise rocprofv3 databases of bench.py runs into the text records kept under profiles/.

  python -m paper_2602_15939_amd.profile_summary trace <results.db> [last_n]
      per-kernel call count and average / total duration (kernel trace); with last_n, also the
      mean duration of the fused push kernel over its last last_n dispatches (the timed steps)
  python -m paper_2602_15939_amd.profile_summary traffic <fetch.db> <write.db> <copy_bytes> \
        [skip [record.json workload source_hash]]
      FETCH_SIZE / WRITE_SIZE per dispatch of the fused push kernel (after the first `skip`
      dispatches), scaled by what the same counters read for the plain device copy of
      copy_bytes in the same run; optionally written as the JSON record bench.py reads
  python -m paper_2602_15939_amd.profile_summary counters <results.db> <kernel substring>
      every counter of a --pmc run for the last dispatch of each kernel whose name contains the
      substring (the last timed step of a bench.py run)
"""
from __future__ import annotations

import collections
import sqlite3
import sys


def kernel_trace(db_path):
    cur = sqlite3.connect(db_path).cursor()
    rows = cur.execute("select name, count(*), avg(end-start), sum(end-start) from kernels "
                       "group by name order by sum(end-start) desc").fetchall()
    return [(n, int(c), a / 1e6, t / 1e6) for n, c, a, t in rows]


def counter_per_dispatch(db_path, counter):
    cur = sqlite3.connect(db_path).cursor()
    rows = cur.execute("select dispatch_id, kernel_name, value from counters_collection "
                       "where counter_name = ?", (counter,)).fetchall()
    per = collections.defaultdict(float)
    names = {}
    for d, k, v in rows:
        per[d] += v
        names[d] = k
    return [(names[d], per[d]) for d in sorted(per)]


def mean_for(rows, pattern):
    vals = [v for k, v in rows if pattern in k]
    return sum(vals) / len(vals) if vals else float("nan"), len(vals)


def dispatches(db_path, pattern):
    cur = sqlite3.connect(db_path).cursor()
    return [(n, (e - s) / 1e6) for n, s, e in cur.execute(
        "select name, start, end from kernels where name like ? order by start", (f"%{pattern}%",))]


def main(argv):
    if argv[0] == "trace":
        print(f"{'kernel':90s} {'calls':>6s} {'avg ms':>10s} {'total ms':>10s}")
        for n, c, a, t in kernel_trace(argv[1])[:25]:
            print(f"{n[:90]:90s} {c:6d} {a:10.4f} {t:10.2f}")
        d = dispatches(argv[1], "gpd_kernel")
        print("gpd_kernel dispatches (ms, in order):", " ".join(f"{t:.4f}" for _, t in d))
        if len(argv) > 2 and d:
            last = [t for _, t in d[-int(argv[2]):]]
            print(f"gpd_kernel mean over the last {len(last)} dispatches (the timed steps): "
                  f"{sum(last) / len(last):.4f} ms")
    elif argv[0] == "traffic":
        fetch, write = counter_per_dispatch(argv[1], "FETCH_SIZE"), counter_per_dispatch(argv[2], "WRITE_SIZE")
        copy_bytes = float(argv[3])
        skip = int(argv[4]) if len(argv) > 4 else 0
        # the calibration copy: the library's plain streaming copy kernel
        cf = max(v for k, v in fetch if "copy_kernel" in k)
        cw = max(v for k, v in write if "copy_kernel" in k)
        gfl = [r for r in fetch if "gpd_kernel" in r[0]][skip:]
        gwl = [r for r in write if "gpd_kernel" in r[0]][skip:]
        gf, nf = mean_for(gfl, "gpd_kernel")
        gw, nw = mean_for(gwl, "gpd_kernel")
        print("gpd_kernel FETCH_SIZE per dispatch:", " ".join(f"{v:.4e}" for _, v in fetch if "gpd" in _))
        print("gpd_kernel WRITE_SIZE per dispatch:", " ".join(f"{v:.4e}" for _, v in write if "gpd" in _))
        sf, sw = copy_bytes / cf, copy_bytes / cw  # bytes per counter unit (KiB nominal)
        print(f"calibration copy: FETCH_SIZE {cf:.4e} WRITE_SIZE {cw:.4e} for {copy_bytes:.4e} B each way")
        print(f"scale: fetch {sf:.2f} B/unit, write {sw:.2f} B/unit")
        print(f"gpd_kernel ({nf} / {nw} dispatches after skipping {skip}): FETCH_SIZE {gf:.4e} -> "
              f"{gf * sf:.4e} B, WRITE_SIZE {gw:.4e} -> {gw * sw:.4e} B, "
              f"total {gf * sf + gw * sw:.4e} B per launch")
        if len(argv) > 6:  # record for bench.py: <record.json> <workload> <source hash>
            import json
            rec = dict(workload=argv[6], source_hash=argv[7], fetch_bytes_per_launch=gf * sf,
                       write_bytes_per_launch=gw * sw, traffic_bytes_per_launch=gf * sf + gw * sw,
                       copy_scale_fetch=sf, copy_scale_write=sw, dispatches=nf)
            with open(argv[5], "w") as fh:
                json.dump(rec, fh, indent=1)
            print("wrote", argv[5])
    elif argv[0] == "counters":
        cur = sqlite3.connect(argv[1]).cursor()
        rows = cur.execute("select dispatch_id, kernel_name, counter_name, value "
                           "from counters_collection").fetchall()
        per = collections.defaultdict(lambda: collections.defaultdict(float))
        names = {}
        for d, k, c, v in rows:
            per[d][c] += v
            names[d] = k
        last = {}
        for d in sorted(per):
            if argv[2] in names[d]:
                last[names[d]] = d
        for k, d in last.items():
            print(k)
            for c, v in sorted(per[d].items()):
                print(f"   {c:28s} {v:.4e}")
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
