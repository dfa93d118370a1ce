"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite) as Markdown.

  python -m paper_2604_26441_amd.profsummary RESULTS_DB [--match NAME --last N] [--solve] [--loop]
  python -m paper_2604_26441_amd.profsummary --counters COUNTER_CSV
  python -m paper_2604_26441_amd.profsummary --traffic FETCH_CSV WRITE_CSV
  python -m paper_2604_26441_amd.profsummary --kuprof FETCH_CSV WRITE_CSV SQ_CSV
  python -m paper_2604_26441_amd.profsummary --l1prof FETCH_CSV WRITE_CSV SQ_CSV

Prints the per-kernel totals (calls, total, average, share) and, with
--match, the average duration of the last N dispatches whose kernel name
contains NAME (for example the back-to-back timing loop of one kernel).
With --solve, also the kernels of the last PCG solve in the trace (from its
k_pcg_init dispatch up to the first later dispatch that is not the
library's, a new k_pcg_init, or a STORE-mode K.u timing launch):
their count, kernel time and first-start to last-end span, per kernel.
With --loop, the same for the last one-launch batch solve, step by step.
With --counters, reads a rocprofv3 --pmc CSV (counter_collection.csv) and
prints, per kernel, the dispatch count and the mean of each counter.
"""
import argparse
import csv
import sqlite3
from collections import defaultdict


def _short(name):
    """Kernel name without namespaces and parameter list."""
    return name.replace("sgmg::", "").replace("(anonymous namespace)::", "").split("(")[0]


def _dispatches(path, counter):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return rows


def traffic(fetch_csv, write_csv, reps, shapes):
    """Per launch shape of the BF16X3 fine K.u (dispatch groups in the order
    the traffic workload ran them), and for the 1 GiB copy: mean FETCH_SIZE
    and WRITE_SIZE (KiB per dispatch), the calibration factors (bytes moved /
    counter bytes, from the copy) and the calibrated HBM bytes per launch."""
    f = _dispatches(fetch_csv, "FETCH_SIZE")
    w = _dispatches(write_csv, "WRITE_SIZE")
    def pick(rows, pred):
        return [float(r["Counter_Value"]) for r in rows if pred(r["Kernel_Name"], int(r["Grid_Size"]))]
    big_copy = lambda n, g: "copyBuffer" in n and g >= 131072
    cf = 1048576.0 / (sum(pick(f, big_copy)) / len(pick(f, big_copy)))
    cw = 1048576.0 / (sum(pick(w, big_copy)) / len(pick(w, big_copy)))
    print(f"calibration: 1 GiB copy, FETCH factor {cf:.4f}, WRITE factor {cw:.4f}")
    ku = lambda n, g: "k_apply_fine_mfma<3," in n and ", 0>" in n
    fk, wk = pick(f, ku), pick(w, ku)
    print("| rows | planes | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | calibrated bytes per launch |")
    print("|---|---|---|---|---|")
    for i, (r, z) in enumerate(shapes):
        a = fk[i * reps:(i + 1) * reps]
        b = wk[i * reps:(i + 1) * reps]
        if len(a) < reps or len(b) < reps:
            break
        fa, wb = sum(a) / reps, sum(b) / reps
        print(f"| {r} | {z} | {fa:.1f} | {wb:.1f} | {round(1024 * (fa * cf + wb * cw))} |")
    # the level-1 stencil applies of the workload: its last reps dispatches
    # (the earlier ones belong to the hierarchy setup)
    st = lambda n, g: "k_stencil_apply_s<double>" in n
    fs, ws = pick(f, st)[-reps:], pick(w, st)[-reps:]
    if len(fs) == reps and len(ws) == reps:
        fa, wb = sum(fs) / reps, sum(ws) / reps
        print()
        print("| kernel | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | calibrated bytes per launch |")
        print("|---|---|---|---|")
        print(f"| `k_stencil_apply_s<double>` level 1 | {fa:.1f} | {wb:.1f} | "
              f"{round(1024 * (fa * cf + wb * cw))} |")


def kuprof(fetch_csv, write_csv, sq_csv, reps, shapes, meshes=(80, 256)):
    """Counter summary of the kuprof workload: per mesh, precision and launch
    shape (dispatch groups of the STORE fine K.u in workload order) the mean
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch), the calibrated HBM bytes
    per launch and their ratio to the algorithmic bytes, and the matrix-core
    busy fraction SQ_VALU_MFMA_BUSY_CYCLES / (32 SQ_BUSY_CYCLES): the first
    sums over the 1024 SIMDs, the second over the 32 shader engines, so the
    ratio is the mean share of a SIMD's cycles its matrix core was busy."""
    f = _dispatches(fetch_csv, "FETCH_SIZE")
    w = _dispatches(write_csv, "WRITE_SIZE")
    mb = _dispatches(sq_csv, "SQ_VALU_MFMA_BUSY_CYCLES")
    sb = _dispatches(sq_csv, "SQ_BUSY_CYCLES")
    def pick(rows, pred):
        return [float(r["Counter_Value"]) for r in rows if pred(r["Kernel_Name"], int(r["Grid_Size"]))]
    big_copy = lambda n, g: "copyBuffer" in n and g >= 131072
    cf = 1048576.0 / (sum(pick(f, big_copy)) / len(pick(f, big_copy)))
    cw = 1048576.0 / (sum(pick(w, big_copy)) / len(pick(w, big_copy)))
    print(f"calibration: 1 GiB copy, FETCH factor {cf:.4f}, WRITE factor {cw:.4f}")
    ku = lambda n, g: "k_apply_fine_mfma<" in n and ", 0>" in n
    fk, wk, mk, sk = pick(f, ku), pick(w, ku), pick(mb, ku), pick(sb, ku)
    print("| mesh | prec | rows | planes | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | calibrated bytes per launch "
          "| / algorithmic | MFMA busy |")
    print("|---|---|---|---|---|---|---|---|---|")
    i = 0
    for n in meshes:
        alg = 2 * 12 * (n + 1) ** 3 + 4 * n ** 3
        for prec in ("bf16", "bf16x3"):
            for r, z in shapes:
                sl = slice(i * reps, (i + 1) * reps)
                i += 1
                a, b, m, q = fk[sl], wk[sl], mk[sl], sk[sl]
                if min(len(a), len(b), len(m), len(q)) < reps:
                    return
                fa, wb = sum(a) / reps, sum(b) / reps
                byts = round(1024 * (fa * cf + wb * cw))
                util = sum(m) / (32.0 * sum(q))
                print(f"| {n}^3 | {prec} | {r} | {z} | {fa:.1f} | {wb:.1f} | {byts} | {byts / alg:.3f} "
                      f"| {util:.3f} |")


L1_SQ = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_VMEM", "SQ_INSTS_LDS",
         "SQ_ACTIVE_INST_VALU", "SQ_WAVE_CYCLES", "SQ_BUSY_CYCLES")


def l1prof(fetch_csv, write_csv, sq_csv, reps, planes=(3, 8), meshes=(80, 128)):
    """Counter summary of the l1prof workload: per mesh and chunk length
    (dispatch groups of the level-1 element-product kernel in workload
    order) the calibrated HBM bytes per launch (as kuprof) and the mean of
    each SQ counter of L1_SQ per dispatch, with the VALU instructions per
    coarse element (per wave, so per 64 elements)."""
    f = _dispatches(fetch_csv, "FETCH_SIZE")
    w = _dispatches(write_csv, "WRITE_SIZE")
    sq = {c: _dispatches(sq_csv, c) for c in L1_SQ}
    def pick(rows, pred):
        return [float(r["Counter_Value"]) for r in rows if pred(r["Kernel_Name"], int(r["Grid_Size"]))]
    big_copy = lambda n, g: "copyBuffer" in n and g >= 131072
    cf = 1048576.0 / (sum(pick(f, big_copy)) / len(pick(f, big_copy)))
    cw = 1048576.0 / (sum(pick(w, big_copy)) / len(pick(w, big_copy)))
    print(f"calibration: 1 GiB copy, FETCH factor {cf:.4f}, WRITE factor {cw:.4f}")
    l1 = lambda n, g: "k_apply_l1_haar<" in n
    fk, wk = pick(f, l1), pick(w, l1)
    sk = {c: pick(v, l1) for c, v in sq.items()}
    print("| mesh | planes | calibrated bytes per launch | " + " | ".join(L1_SQ) +
          " | VALU instructions per coarse element x 64 |")
    print("|---|---|---|" + "---|" * len(L1_SQ) + "---|")
    i = 0
    for n in meshes:
        ne = (n // 2) ** 3
        for z in planes:
            sl = slice(i * reps, (i + 1) * reps)
            i += 1
            a, b = fk[sl], wk[sl]
            if min(len(a), len(b)) < reps or any(len(v[sl]) < reps for v in sk.values()):
                return
            byts = round(1024 * (sum(a) / reps * cf + sum(b) / reps * cw))
            means = [sum(sk[c][sl]) / reps for c in L1_SQ]
            print(f"| {n}^3 | {z} | {byts} | " + " | ".join(f"{m:.0f}" for m in means) +
                  f" | {means[1] * 64 / ne:.0f} |")


def counters(path):
    acc = defaultdict(lambda: defaultdict(list))
    with open(path) as fh:
        for row in csv.DictReader(fh):
            name = _short(row.get("Kernel_Name", ""))
            acc[name][row["Counter_Name"]].append(float(row["Counter_Value"]))
    cols = sorted({c for k in acc.values() for c in k})
    print("| kernel | dispatches | " + " | ".join(f"mean {c}" for c in cols) + " |")
    print("|---|---|" + "---|" * len(cols))
    for name, byc in acc.items():
        nd = max(len(v) for v in byc.values())
        vals = [sum(byc[c]) / len(byc[c]) if byc[c] else float("nan") for c in cols]
        print(f"| `{name}` | {nd} | " + " | ".join(f"{v:.1f}" for v in vals) + " |")


def last_solve(c, marker="k_apply_fine_sf64<3>"):
    rows = list(c.execute("select name, start, end from kernels order by start"))
    starts = [i for i, r in enumerate(rows) if "k_pcg_init" in r[0]]
    if not starts:
        return
    i0 = starts[-1]
    seg = rows[i0:]
    # the solve ends before the first kernel that is not the library's (the
    # caller's own work), a new solve, or a timing loop of STORE K.u
    end = len(seg)
    for k, r in enumerate(seg[1:], 1):
        if ("sgmg::" not in r[0] and "rocclr" not in r[0]) or "k_pcg_init" in r[0] or \
                "mfma<3, 4, 0>" in r[0] or "mfma<3, 8, 0>" in r[0]:
            end = k
            break
    seg = seg[:end]
    busy = sum(e - s for _, s, e in seg)
    span = seg[-1][2] - seg[0][1]
    tot = defaultdict(lambda: [0, 0])
    for n, s, e in seg:
        k = _short(n)
        tot[k][0] += 1
        tot[k][1] += e - s
    print(f"\nLast solve: {len(seg)} kernels, {busy / 1e3:.0f} us of kernel time in "
          f"{span / 1e3:.0f} us from the first kernel's start to the last one's end.\n")
    print("| kernel | calls | total (us) | average (us) | share of kernel time |")
    print("|---|---|---|---|---|")
    for k, (n, t) in sorted(tot.items(), key=lambda kv: -kv[1][1]):
        print(f"| `{k}` | {n} | {t / 1e3:.1f} | {t / n / 1e3:.2f} | {100 * t / busy:.1f}% |")
    # per PCG iteration: the kernel time from one outer K p dispatch (marker)
    # to the next; the last one runs to the end of the solve and also holds
    # the final true-residual check
    kp = [i for i, r in enumerate(seg) if marker in r[0]]
    if len(kp) > 1:
        its = [sum(e - s for _, s, e in seg[a:b]) / 1e3 for a, b in zip(kp, kp[1:])]
        print(f"\nKernel time per PCG iteration (from one `{_short(marker)}` dispatch to the next): "
              + ", ".join(f"{x:.1f}" for x in its) + f" us; mean {sum(its) / len(its):.1f} us. "
              f"Before the first: {sum(e - s for _, s, e in seg[:kp[0]]) / 1e3:.1f} us; "
              f"from the last to the end: {sum(e - s for _, s, e in seg[kp[-1]:]) / 1e3:.1f} us.")


def last_loop(c, every=10):
    """The last one-launch batch solve in the trace (from its k_bs_loop_init
    to the k_bs_final_rel that ends the launch): kernel count, kernel time
    and span, then per PCG step (the dispatches up to and including that
    step's k_bs_decide_check) the dispatch count, kernel time and span for
    every `every`-th step and the last one."""
    rows = list(c.execute("select name, start, end from kernels order by start"))
    starts = [i for i, r in enumerate(rows) if "k_bs_loop_init" in r[0]]
    if not starts:
        return
    seg = rows[starts[-1]:]
    ends = [i for i, r in enumerate(seg) if "k_bs_final_rel" in r[0]]
    seg = seg[:ends[0] + 1]
    busy = sum(e - s for _, s, e in seg)
    print(f"\nLast one-launch solve: {len(seg)} kernels, {busy / 1e3:.0f} us of kernel time in "
          f"{(seg[-1][2] - seg[0][1]) / 1e3:.0f} us from the first kernel's start to the last "
          "one's end.\n")
    cuts = [i for i, r in enumerate(seg) if "k_bs_decide_check" in r[0]]
    first = [i for i, r in enumerate(seg) if "k_bs_decide_start" in r[0]][0]
    bounds = [first] + cuts
    print("| step | dispatches | kernel time (us) | span (us) | mean dispatch (us) |")
    print("|---|---|---|---|---|")
    for k in range(1, len(bounds)):
        if k % every and k != 1 and k != len(bounds) - 1:
            continue
        st = seg[bounds[k - 1] + 1:bounds[k] + 1]
        kt = sum(e - s for _, s, e in st)
        print(f"| {k} | {len(st)} | {kt / 1e3:.1f} | {(st[-1][2] - st[0][1]) / 1e3:.1f} | "
              f"{kt / len(st) / 1e3:.2f} |")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db", nargs="?")
    ap.add_argument("--counters", default=None)
    ap.add_argument("--traffic", nargs=2, default=None, metavar=("FETCH_CSV", "WRITE_CSV"))
    ap.add_argument("--kuprof", nargs=3, default=None, metavar=("FETCH_CSV", "WRITE_CSV", "SQ_CSV"))
    ap.add_argument("--l1prof", nargs=3, default=None, metavar=("FETCH_CSV", "WRITE_CSV", "SQ_CSV"))
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--match", default=None)
    ap.add_argument("--last", type=int, default=200)
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--solve", action="store_true")
    ap.add_argument("--loop", action="store_true")
    a = ap.parse_args()
    if a.counters:
        counters(a.counters)
        return
    # the shape order of experiments.TRAFFIC_SHAPES
    shapes = [(r, z) for r in (4, 8) for z in (2, 4, 8, 16, 32)]
    if a.traffic:
        traffic(a.traffic[0], a.traffic[1], a.reps, shapes)
        return
    if a.l1prof:
        l1prof(a.l1prof[0], a.l1prof[1], a.l1prof[2], a.reps)
        return
    if a.kuprof:
        kuprof(a.kuprof[0], a.kuprof[1], a.kuprof[2], a.reps, shapes)
        return
    c = sqlite3.connect(a.db)
    rows = list(c.execute("select name, total_calls, total_duration, average, percentage "
                          "from top_kernels"))
    print("| kernel | calls | total (ms) | average (us) | share |")
    print("|---|---|---|---|---|")
    for name, calls, tot, avg, pct in rows[: a.top]:
        short = _short(name)
        print(f"| `{short}` | {calls} | {tot / 1e3:.3f} | {avg:.3f} | {pct:.1f}% |")
    if a.solve:
        last_solve(c)
    if a.loop:
        last_loop(c)
    if a.match:
        durs = [r[0] for r in c.execute(
            "select duration from kernels where name like ? order by start", (f"%{a.match}%",))]
        last = durs[-a.last:]
        if last:
            print(f"\nLast {len(last)} dispatches matching `{a.match}`: average "
                  f"{sum(last) / len(last) / 1e3:.3f} us, min {min(last) / 1e3:.3f} us, "
                  f"max {max(last) / 1e3:.3f} us")


if __name__ == "__main__":
    main()
