"""Autotuner for the stage-5 tiles (argument marshalling and timing over the C ABI).

The stage-5 kernels have two launch parameters that the best choice of depends on the
problem size and on the chip: the rows per workgroup (rb 32-row blocks per wave, FP32 and
BF16 kernels) and how the l-range is split across workgroups (split count for one
problem, l-points per split for a batch).  The tuner times every candidate with HIP
events on the device (kl_profile_* for one problem, events around the graph replay for a
batch), keeps the fastest, and caches it in a JSON file keyed by

    (GPU architecture, dimension, covariance kind, precision, padded grid size)

for single problems (plus the objective when it is the whole apply), and by
(architecture, dimension, precision, batch signature) for batches.  The objective of a
single problem is the stage-5 kernel alone (`objective="stage5"`, the default) or the whole
apply of a 32-column block (`objective="apply"`): the fused backward Kronecker launch adds
the stage-5 split partials, so fewer splits can make the apply faster even when the kernel
alone is not.  With the whole apply as the objective the tuner also chooses between the
fused Kronecker launches (first two directions of each side in one launch, the backward
one adding the split partials) and one launch per direction (split partials added by their
own pass), re-scanning the split count for the latter.  For FP64, BF16 and BF16x3 it then
times the symmetric form of stage 5 (kl_stage5_symmetric) on the same objective and keeps it
when it is faster.  Cached settings are applied with
`apply_cached`; a problem without an entry of its own takes the entry of the nearest
tuned padded size within 25 % (same architecture, dimension, kind, precision, objective):
the size buckets of the cache.  The cache file is $KL_TUNE_CACHE, else
~/.cache/paper_2011_13861_amd/stage5_tune.json.
"""

import hashlib
import json
import os


SYMMETRIC_PRECISIONS = ("f64", "bf16", "bf16x3")     # stage 5 has a symmetric form


def cache_path():
    return os.environ.get("KL_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_2011_13861_amd", "stage5_tune.json")


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def arch():
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def _padded(nt):
    return (nt + 255) // 256 * 256


def problem_key(G, kind, precision, objective="stage5", arch_name=None):
    parts = [arch_name or arch(), "d%d" % G.d, kind, precision, "Np%d" % _padded(G.Nt)]
    if objective != "stage5":
        parts.append(objective)
    return "|".join(parts)


def lookup(data, key, bucket=0.25):
    """The cache entry of `key`, else the one whose padded size is nearest to the key's
    among entries that differ from it in the size only, if within `bucket` (relative)."""
    if key in data:
        return data[key]
    parts = key.split("|")
    i = next(j for j, p in enumerate(parts) if p.startswith("Np"))
    np0 = int(parts[i][2:])
    best = None
    for k, e in data.items():
        q = k.split("|")
        if len(q) != len(parts) or q[:i] + q[i + 1:] != parts[:i] + parts[i + 1:] or not q[i].startswith("Np"):
            continue
        d = abs(int(q[i][2:]) - np0) / np0
        if d <= bucket and (best is None or d < best[0]):
            best = (d, e)
    return best[1] if best else None


def batch_key(B, kinds, precision):
    sig = hashlib.sha1(json.dumps([[_padded(nt), k] for nt, k in zip(B.Nt, kinds)]).encode()).hexdigest()[:16]
    return "|".join([arch(), "batch", precision, "n%d" % B.n, sig])


def _time_problem(G, precision, reps, nvec=32):
    import torch
    yin = torch.randn((nvec, G.Nt), dtype=torch.float64, device="cuda").T
    z = torch.empty((nvec, G.Nt), dtype=torch.float64, device="cuda").T
    for _ in range(3):
        G.stage5(yin, z, precision)
    torch.cuda.synchronize()
    G.profile_enable(True)
    for _ in range(reps):
        G.stage5(yin, z, precision)
    torch.cuda.synchronize()
    cnt, ms = G.profile_read()[precision]
    G.profile_enable(False)
    return ms / max(cnt, 1) * 1e3


def _time_apply(G, precision, reps, nvec=32):
    import torch
    x = torch.randn((nvec, G.N), dtype=torch.float64, device="cuda").T
    y = torch.empty((nvec, G.N), dtype=torch.float64, device="cuda").T
    for _ in range(3):
        G.apply(x, y, precision)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        G.apply(x, y, precision)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps * 1e3


def pick(timed, tie=0.015):
    """The setting to keep among timed (rb, nsplit, us) candidates: within `tie` of the
    fastest (timing noise), the one whose split partials cost the least HBM traffic: a
    split count that is a multiple of 8 (each XCD then reads only its own columns of the
    stage-5 input), then the fewest splits (fewer partials to write and add), then the
    fastest."""
    fastest = min(t[2] for t in timed)
    near = [t for t in timed if t[2] <= fastest * (1.0 + tie)]
    return min(near, key=lambda t: (t[1] % 8 != 0 and t[1] != 1, t[1], t[2]))


def tune_problem(G, kind, precisions=("f32",), reps=20, max_split=64, path=None, verbose=False,
                 objective="stage5"):
    """Searches (rb, nsplit) for each precision on problem G (covariance `kind`), sets
    the best for the objective ("stage5": the kernel alone; "apply": the whole apply of
    a 32-column block), records it in the cache and returns {precision: (rb, nsplit, us)}."""
    if objective not in ("stage5", "apply"):
        raise ValueError("objective must be 'stage5' or 'apply'")
    timer = _time_problem if objective == "stage5" else _time_apply
    path = path or cache_path()
    data = _load(path)
    out = {}

    def scan(prec, rbs):
        timed = []
        for rb in rbs:
            _, auto = G.stage5_config(prec, rb=rb, nsplit=0)
            cands = sorted({auto, 1} | set(range(2, max_split + 1, 1 if max_split <= 24 else 2)))
            for ns in cands:
                rbe, nse = G.stage5_config(prec, rb=rb, nsplit=ns)
                if nse != ns and ns != auto:
                    continue                      # capped: same as a smaller candidate
                us = timer(G, prec, reps)
                if verbose:
                    print("tune", prec, rbe, nse, "%.1f us" % us)
                timed.append((rbe, nse, us))
        return pick(timed)

    for prec in precisions:
        rbs = [2] if prec == "f64" else ([1, 2, 4, 8] if prec == "f32" else [1, 2, 4])
        fused = G.apply_config(True)
        best = scan(prec, rbs)
        fuse = fused
        if objective == "apply" and fused:
            # one launch per direction, with the tile height found above
            G.apply_config(False)
            alt = scan(prec, [best[0]])
            if alt[2] < best[2] * (1.0 - 0.015):
                best, fuse = alt, False
            G.apply_config(fuse)
        G.stage5_config(prec, rb=best[0], nsplit=best[1])
        sym = False
        if prec in SYMMETRIC_PRECISIONS:
            # the symmetric form (half the kernel evaluations, partial sums in a fixed order)
            # against the best plain setting, on the same objective
            G.stage5_symmetric(True, precision=prec)
            us = timer(G, prec, reps)
            if verbose:
                print("tune", prec, "symmetric", "%.1f us" % us)
            sym = us < best[2] * (1.0 - 0.015)
            if sym:
                best = (best[0], best[1], us)
            else:
                G.stage5_symmetric(False, precision=prec)
        data[problem_key(G, kind, prec, objective)] = {"rb": best[0], "nsplit": best[1], "us": best[2],
                                                        "fuse": bool(fuse), "sym": bool(sym)}
        out[prec] = best
    _store(path, data)
    return out


def tune_batch(B, kinds, precision="f32", reps=10, path=None, verbose=False):
    """Searches (rb, l-points per split) of the batched stage-5 kernel by timing whole
    graph replays (32 columns per problem); sets and records the best."""
    import torch
    path = path or cache_path()
    data = _load(path)
    x = torch.randn(B.Ntot * 32, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    rbs = [2] if precision == "f64" else [2, 4]
    best = None
    for rb in rbs:
        for lc in (0, 512, 1024, 2048, 4096, 8192, 16384):
            B.config(precision, rb=rb, lchunk=lc)
            for _ in range(2):
                B.apply(x, y, 32, precision)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                B.apply(x, y, 32, precision)
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) / reps * 1e3
            if verbose:
                print("tune batch", precision, rb, lc, "%.1f us" % us)
            if best is None or us < best[2]:
                best = (rb, lc, us)
    B.config(precision, rb=best[0], lchunk=best[1])
    data[batch_key(B, kinds, precision)] = {"rb": best[0], "lchunk": best[1], "us": best[2]}
    _store(path, data)
    return best


def apply_cached(G, kind, precision, path=None, objective="stage5"):
    """Sets the cached setting for G (its own, else its size bucket's), if any; returns it
    (or None)."""
    e = lookup(_load(path or cache_path()), problem_key(G, kind, precision, objective))
    if e:
        G.stage5_config(precision, rb=e["rb"], nsplit=e["nsplit"])
        if "fuse" in e:
            G.apply_config(e["fuse"])
        if precision in SYMMETRIC_PRECISIONS and "sym" in e:
            G.stage5_symmetric(e["sym"], precision=precision)
    return e


def apply_cached_batch(B, kinds, precision, path=None):
    e = _load(path or cache_path()).get(batch_key(B, kinds, precision))
    if e:
        B.config(precision, rb=e["rb"], lchunk=e["lchunk"])
    return e
