"""Short text summaries of rocprofv3 CSV output (kernel statistics and HBM
traffic counters), for keeping beside the measurements they back.

    python -m paper_2008_06972_amd.profile_summary stats DIR NAME OUT "COMMAND"
    python -m paper_2008_06972_amd.profile_summary traffic DIR FETCH WRITE \
        COPY_FETCH COPY_WRITE COPY_BYTES OUT "COMMANDS"

``stats`` turns ``DIR/NAME_kernel_stats.csv`` into a table.  ``traffic``
reads the per-dispatch FETCH_SIZE and WRITE_SIZE counters (KiB) of the
batched encoder's kernels and of a plain device copy of COPY_BYTES bytes
(read once, written once); the copy's readings give the scale from counter
units to bytes, which is applied to every kernel.  The result is JSON keyed
by launch kind (count, scatter, keyimage, net, key, pred, finish, ...) with
the hash of the kernel sources it was taken on: bytes per pass of the batch
graph for its kinds (a pass launches binning twice, for key and for
predicted frames), per dispatch for the others.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

KINDS = (("k_batch_bin", "bin"), ("k_batch_count", "count"), ("k_batch_scatter", "scatter"), ("k_batch_keyimage", "keyimage"),
         ("k_net_", "net"), ("k_batch_key", "key"),
         ("k_batch_pred", "pred"), ("k_batch_finish", "finish"), ("k_batch_offsets", "offsets"),
         ("k_batch_reset", "reset"), ("k_pack_", "pack"), ("k_decode", "decode"))


# launch kinds of the batch graph: their traffic is given per pass
PASS_KINDS = ("bin", "count", "scatter", "keyimage", "net", "key", "pred", "finish", "offsets", "reset")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2008_06972_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, fn), "rb") as f:
            h.update(fn.encode() + f.read())
    return h.hexdigest()[:16]


def kind_of(name: str):
    for key, kind in KINDS:
        if key in name:
            return kind
    return None


def short(name: str, n: int = 60) -> str:
    name = name.replace("(anonymous namespace)::", "").split("(")[0]
    return name if len(name) <= n else name[: n - 3] + "..."


def stats(d, name, out, command):
    rows = list(csv.DictReader(open(os.path.join(d, f"{name}_kernel_stats.csv"))))
    lines = [f"# rocprofv3 kernel statistics", f"command: {command}", "",
             f"{'kernel':60s} {'calls':>7s} {'avg us':>10s} {'min us':>10s} {'max us':>10s} {'total %':>8s}"]
    for r in rows:
        lines.append(f"{short(r['Name']):60s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.2f} "
                     f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} "
                     f"{float(r['Percentage']):8.2f}")
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counter(path, counter):
    """{kernel name: [values per dispatch]} of one counter."""
    out = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def traffic(d, fetch, write, copy_fetch, copy_write, copy_bytes, out, command):
    cf = _counter(os.path.join(d, f"{copy_fetch}_counter_collection.csv"), "FETCH_SIZE")
    cw = _counter(os.path.join(d, f"{copy_write}_counter_collection.csv"), "WRITE_SIZE")

    def copy_value(m):
        # the copy is the only kernel of that size: take the largest reading
        return max(max(v) for v in m.values())
    kib = copy_bytes / 1024.0
    f_fetch = kib / copy_value(cf)
    f_write = kib / copy_value(cw)
    bf = _counter(os.path.join(d, f"{fetch}_counter_collection.csv"), "FETCH_SIZE")
    bw = _counter(os.path.join(d, f"{write}_counter_collection.csv"), "WRITE_SIZE")
    # a pass of the batch graph launches the predicted-frame encoder once;
    # kinds launched several times per pass (binning of key and predicted
    # frames) are summed over the pass
    passes = {m: max(1, sum(len(v) for n, v in b.items() if kind_of(n) == "pred")) for m, b in (("f", bf), ("w", bw))}
    kernels = {}
    for name in sorted(set(bf) | set(bw)):
        kind = kind_of(name)
        if kind is None:
            continue
        fv, wv = bf.get(name, []), bw.get(name, [])
        if kind in PASS_KINDS:
            fb = sum(fv) / passes["f"] * 1024.0 * f_fetch
            wb = sum(wv) / passes["w"] * 1024.0 * f_write
        else:
            fb = sum(fv) / max(1, len(fv)) * 1024.0 * f_fetch
            wb = sum(wv) / max(1, len(wv)) * 1024.0 * f_write
        k = kernels.setdefault(kind, {"kernels": [], "fetch_bytes": 0.0, "write_bytes": 0.0})
        k["kernels"].append(short(name))
        k["fetch_bytes"] += fb
        k["write_bytes"] += wb
    for kind, k in kernels.items():
        k["bytes_per_launch"] = k["fetch_bytes"] + k["write_bytes"]
        k["per"] = "pass" if kind in PASS_KINDS else "dispatch"
    res = {"source_hash": kernel_source_hash(), "command": command, "copy_bytes": copy_bytes,
           "scale_fetch": f_fetch, "scale_write": f_write, "kernels": kernels}
    json.dump(res, open(out, "w"), indent=1)
    print(json.dumps(res, indent=1))


def main(argv):
    if argv[0] == "stats":
        stats(argv[1], argv[2], argv[3], argv[4])
    elif argv[0] == "traffic":
        traffic(argv[1], argv[2], argv[3], argv[4], argv[5], int(argv[6]), argv[7], argv[8])
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
