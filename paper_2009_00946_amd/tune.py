"""Launch-shape cache around the library's autotuner (fewha_autotune).

The tuner itself is native: it times the stage kernels of a bound plan for every valid launch
shape (forward-DWT split, fine tile size, XCD chunks) and keeps the fastest.  This module keeps
its results in a JSON file keyed by everything the timing depends on (geometry, precision, frames
per launch, device architecture and compute-unit count), so a plan of a known geometry gets its
shapes without timing again.

    from paper_2009_00946_amd import fewha, tune
    P = fewha.Plan(cfg, max_batch=32)
    shapes = tune.tuned(P)          # from the cache, else autotuned and stored
"""
import hashlib
import json
import os

CACHE_ENV = "FEWHA_TUNE_CACHE"


def default_cache():
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache", "fewha", "tuning.json")


def geometry_key(cfg, precision, nbatch, device):
    """Hash of the plan inputs that set the kernels' launch grids and costs."""
    geo = {"D": cfg["D"], "obstruction": cfg.get("obstruction", 0.0), "J": cfg["J"],
           "wfs": [[w["n_sub"], w["theta_x"], w["theta_y"], w["gs_height"]] for w in cfg["wfs"]],
           "layers": [[l["height"], l["spacing"], l["n"]] for l in cfg["layers"]],
           "dms": [[d["height"], d["pitch"], d["n_act"]] for d in cfg["dms"]],
           "precision": precision, "nbatch": int(nbatch), "device": device}
    return hashlib.sha256(json.dumps(geo, sort_keys=True).encode()).hexdigest()[:32]


def device_id(device):
    """Architecture and compute-unit count of a device (its marketing name can differ between
    runtimes, e.g. under a profiler, while the tuned shapes still apply)."""
    import torch
    pr = torch.cuda.get_device_properties(device)
    return "%s/%dcu" % (getattr(pr, "gcnArchName", pr.name).split(":")[0], pr.multi_processor_count)


def _read(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tuned(P, nbatch=None, cache=None, retune=False):
    """Launch shapes for plan P (set on it): cached for its key, else fewha_autotune's (which resets
    the plan's chain state) stored in the cache.  Returns {"tuning", "us", "key", "cached"}."""
    import torch
    nb = P.max_batch if nbatch is None else int(nbatch)
    path = cache or default_cache()
    key = geometry_key(P.cfg, P.precision, nb, device_id(P.device))
    db = _read(path)
    if key in db and not retune:
        rec = db[key]
        P.set_tuning(rec["tuning"])
        return dict(rec, key=key, cached=True)
    tuning, us = P.autotune(nb)
    rec = {"tuning": tuning, "us": {k: round(v, 3) for k, v in us.items()}, "config": P.cfg.get("name", "")}
    db = _read(path)
    db[key] = rec
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return dict(rec, key=key, cached=False)
