"""HBM traffic per launch of a kernel from two rocprofv3 counter runs.

Usage:
    python -m paper_1407_4524_amd.hbm_traffic FETCH.csv WRITE.csv KERNEL_PREFIX \
        COPY_BYTES OUT.json [--note TEXT]

FETCH.csv and WRITE.csv are the ``*_counter_collection.csv`` files of two
``rocprofv3 --pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs of the same command
(counters in KiB per dispatch). That command must also launch the library's
plain copy kernel (``lbm::k_copy``, see lbm_copy) moving COPY_BYTES in total,
half read and half written: each counter is scaled by what it reads for that
copy against the bytes the copy is known to move. On gfx950 the write
counter reads the copy's bytes exactly (scale 1.000) and the fetch counter
half of them (0.500): FETCH_SIZE prices every read request that is not a
32-byte one at 64 bytes, while the L2 fetches whole 128-byte lines per
request (TCC_EA0_RDREQ_sum x 128 equals the copy's source bytes). The
kernel is the one whose name starts with KERNEL_PREFIX and whose grid is the
most frequent among its dispatches.
"""
import argparse
import collections
import csv
import hashlib
import json
import os

COPY_KERNEL = "void lbm::k_copy"
HERE = os.path.dirname(os.path.abspath(__file__))


def kernel_source_hash():
    """Hash of the sources of the stream-collide kernel (sweep.hpp and the
    layout headers it reads): a summary is only valid for the kernel it was
    taken on."""
    h = hashlib.sha256()
    for f in ("sweep.hpp", "lattice.hpp", "geom.hpp"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def per_dispatch(path, counter):
    """{(kernel name, grid): [KiB per dispatch]} of one counter"""
    out = collections.defaultdict(list)
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                out[(r["Kernel_Name"], r["Grid_Size"])].append(float(r["Counter_Value"]))
    return out


def pick(d, prefix):
    cands = {k: v for k, v in d.items() if k[0].startswith(prefix)}
    if not cands:
        raise SystemExit(f"no dispatch of a kernel starting with {prefix!r}")
    k = max(cands, key=lambda k: len(cands[k]))
    v = cands[k]
    return k, sum(v) / len(v), len(v)


def summarize(fetch_csv, write_csv, prefix, copy_bytes):
    f = per_dispatch(fetch_csv, "FETCH_SIZE")
    w = per_dispatch(write_csv, "WRITE_SIZE")
    (kname, grid), kf, nf = pick(f, prefix)
    _, kw, nw = pick(w, prefix)
    _, cf, _ = pick(f, COPY_KERNEL)
    _, cw, _ = pick(w, COPY_KERNEL)
    half = copy_bytes / 2
    fetch_scale = cf * 1024 / half  # counter KiB*1024 per byte really read
    write_scale = cw * 1024 / half
    read = kf * 1024 / fetch_scale
    written = kw * 1024 / write_scale
    return dict(kernel=kname, grid=int(grid), dispatches=[nf, nw], fetch_kib_per_dispatch=round(kf, 1),
                write_kib_per_dispatch=round(kw, 1), copy_bytes=copy_bytes, copy_fetch_kib=round(cf, 1),
                copy_write_kib=round(cw, 1), fetch_scale=round(fetch_scale, 4), write_scale=round(write_scale, 4),
                hbm_read_bytes_per_launch=round(read), hbm_write_bytes_per_launch=round(written),
                hbm_bytes_per_launch=round(read + written), kernel_source_sha256_16=kernel_source_hash())


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("fetch_csv")
    ap.add_argument("write_csv")
    ap.add_argument("kernel_prefix")
    ap.add_argument("copy_bytes", type=int)
    ap.add_argument("out_json")
    ap.add_argument("--note", default="")
    a = ap.parse_args()
    rec = summarize(a.fetch_csv, a.write_csv, a.kernel_prefix, a.copy_bytes)
    rec["note"] = a.note
    with open(a.out_json, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
