"""Helpers of the GPU-vs-oracle parity tests.

The oracle always computes from the seeded inputs and its own fit; the GPU index is built
from the oracle's artifacts (ddc_import) so both sides search the same lists, stored
values and correction table.  Nothing computed by the GPU is fed back into the oracle.
"""
import functools

import numpy as np

import oracle as O
import synthdata

TOL = 1e-4   # relative: ids may differ only near a decision threshold; dists within this


@functools.lru_cache(maxsize=None)
def workload(name, n=None, nq=None, n_calib=None, n_val=None, D=None):
    w = synthdata.make_workload(name, n=n, nq=nq, n_calib=n_calib, n_val=n_val)
    if D is not None:          # ragged dimensionality: keep the leading D coordinates
        w = dict(w)
        for k in ("base", "queries", "calib", "val"):
            w[k] = np.ascontiguousarray(w[k][:, :D])
    return w


@functools.lru_cache(maxsize=None)
def oracle_index(name="gauss128", nlist=64, storage="f32", delta_d=32, B=256, n=None, n_calib=None,
                 calib_k=10, calib_nprobe=8, D=None, kmeans_iters=25, seed=7, fp8_lead=0, pq_m=0,
                 calib_k_extra=(), L=0):
    w = workload(name, n=n, n_calib=n_calib, D=D)
    ix = O.fit(w["base"], w["calib"], nlist=nlist, delta_d=delta_d, storage=storage,
               kmeans_iters=kmeans_iters, calib_k=calib_k, calib_nprobe=calib_nprobe, B=B, L=L, seed=seed,
               fp8_lead=fp8_lead, pq_m=pq_m, pq_iters=8, calib_k_extra=calib_k_extra)
    # centroids handed to the GPU in float32: the oracle uses the same float32 values
    ix["centroids"] = ix["centroids"].astype(np.float32).astype(np.float64)
    return ix


def artifacts(ix, with_table=True):
    art = dict(mu=ix["mu"], R=ix["R"], lam=ix["lam"], centroids=ix["centroids"].astype(np.float32),
               assign=ix["assign"].astype(np.int32), y=ix["Y"].astype(np.float32),
               storage=ix["storage"], delta_d=ix["delta_d"], block_b=ix["B"], lag_l=ix.get("L", 0))
    if ix.get("pre") is not None:
        art["fp8_lead_dims"] = ix["pre"]["lead"]
    if ix.get("pq") is not None:
        art.update(pq_perm=ix["pq"]["perm"], pq_books=ix["pq"]["books"].astype(np.float32))
    if with_table:
        art.update(m=ix["m"], resid=ix["G"])
        if ix.get("pq") is not None:
            t0 = ix["pq_tab"]
            art.update(pq_m1=t0["m1"], pq_m3=t0["m3"], pq_resid=t0["G"][:, 0])
        if ix.get("tables"):
            art["tables"] = [dict(kc=t["kc"], m=t["m"], resid=t["G"]) for t in ix["tables"]]
            if ix.get("pq") is not None:
                for d, t in zip(art["tables"], ix["tables"]):
                    d.update(pq_m1=t["pq"]["m1"], pq_m3=t["pq"]["m3"], pq_resid=t["pq"]["G"][:, 0])
    return art


def check_search(gpu_ids, gpu_d, ora, ix, tol=TOL, k=None):
    """Per query: ids identical to the oracle's unless the oracle logged a decision within
    `tol` (relative) of its threshold; every GPU distance within `tol` of the FP64 distance of
    the returned stored vector; results sorted and padded.  Returns a summary dict."""
    nq = gpu_ids.shape[0]
    same = excused = 0
    bad = []
    Y = ix["Y"]
    for qi in range(nq):
        gi, gd = gpu_ids[qi], gpu_d[qi].astype(np.float64)
        oi, od = ora["ids"][qi], ora["dists"][qi]
        valid = gi >= 0
        # padding layout identical to the oracle's (same candidate counts)
        if not np.array_equal(valid, oi >= 0):
            bad.append((qi, "padding"))
            continue
        if np.any(np.isfinite(gd[~valid])) or np.any(gi[~valid] != -1):
            bad.append((qi, "pad values"))
            continue
        if valid.any():
            exact = O.sq_dist_direct(Y[gi[valid]], ora["qrot"][qi])
            if not np.allclose(gd[valid], exact, rtol=tol, atol=tol * max(1e-30, float(exact.max()))):
                bad.append((qi, "distance"))
                continue
            if np.any(np.diff(gd[valid]) < 0):
                bad.append((qi, "order"))
                continue
            if len(set(gi[valid].tolist())) != int(valid.sum()):
                bad.append((qi, "duplicate id"))
                continue
        if np.array_equal(gi, oi):
            same += 1
            if not np.allclose(gd[valid], od[valid], rtol=tol):
                bad.append((qi, "distance vs oracle"))
        elif ora["margin"][qi] < tol:
            excused += 1
        else:
            bad.append((qi, f"ids differ, oracle margin {ora['margin'][qi]:.3g}"))
    return dict(nq=nq, same=same, excused=excused, bad=bad)
