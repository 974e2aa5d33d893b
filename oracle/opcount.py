"""Operation counts of the step oracle -- TEST AND MEASUREMENT INFRASTRUCTURE.

``opcount.cpp`` compiles ``nyx_oracle.c`` unchanged with a counting number
type, so every +, -, *, / and sqrt of the published algorithm, as the oracle
evaluates it on given data, is counted against its stage (O1 ... O13) and,
inside the two-shock solver, against the Newton iterations.  Comparisons,
fabs, min/max and selects are not flops (counted apart as comparisons).

Run as a script, it writes ``profiles/opcounts_step.json``: the flops per
work unit of each stage kernel of the HIP path (the unit each kernel's grid
runs over), measured on samples of the benchmark workloads.  The benchmark
reads that table for the algorithmic flops of its roofline figures; nothing
in the HIP library reads it.
"""
from __future__ import annotations

import ctypes
import json
import os
import subprocess
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
_SO = os.path.join(_HERE, "libnyxopcount.so")
_SRC = os.path.join(_HERE, "opcount.cpp")
TABLE = os.path.join(_ROOT, "profiles", "opcounts_step.json")

# the oracle's own flags, as C++
CXXFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared", "-std=c++17", "-w"]

STAGE_NAMES = {1: "prim", 2: "flat", 3: "trace", 4: "riem0", 5: "riem1", 6: "riem2",
               7: "update", 8: "cfl"}
OPS = ("add", "mul", "div", "sqrt", "cmp")
NSTAGE = 9


def build(force: bool = True) -> str:
    if not force and os.path.exists(_SO):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.run(["g++"] + CXXFLAGS + ["-I", _HERE, "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        D = ctypes.POINTER(ctypes.c_double)
        i, d, v = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        L.nyxo_opcount_reset.argtypes = []
        L.nyxo_opcount_read.argtypes = [ctypes.POINTER(ctypes.c_longlong)]
        L.nyxo_opcount_step.argtypes = [v, i, i, i, i, D, D, d, d, d, d, D,
                                        ctypes.POINTER(ctypes.c_longlong)]
        L.nyxo_opcount_step.restype = i
        L.nyxo_opcount_dt.argtypes = [v, i, i, i, i, D, d, d, d, D]
        L.nyxo_opcount_dt.restype = i
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _read():
    buf = (ctypes.c_longlong * (NSTAGE * 2 * len(OPS)))()
    lib().nyxo_opcount_read(buf)
    return np.array(buf[:], dtype=np.int64).reshape(NSTAGE, 2, len(OPS))


def _params(params):
    import oracle
    return (params or oracle.Params()).c()


def count_step(state, grav, ng, dt, dx, a_old, a_new, params=None):
    """One oracle step under the counting type.  Returns (new_state, stats,
    counts) with counts[stage][iter][op] (iter 1 = inside a Newton iteration
    of the two-shock solver)."""
    state = np.ascontiguousarray(state, dtype=np.float64)
    grav = np.ascontiguousarray(grav, dtype=np.float64)
    nz, ny, nx = (s - 2 * ng for s in state.shape[1:])
    out = state.copy()
    st = (ctypes.c_longlong * 8)()
    prm = _params(params)
    L = lib()
    L.nyxo_opcount_reset()
    rc = L.nyxo_opcount_step(ctypes.byref(prm), nx, ny, nz, ng, _ptr(state), _ptr(grav), dt, dx,
                             a_old, a_new, _ptr(out), st)
    if rc != 0:
        raise ValueError("nyxo_opcount_step: bad arguments")
    import oracle
    stats = dict(zip(oracle.STATS_FIELDS, st[:]))
    return out, stats, _read()


def count_dt(state, ng, a, dx, cfl, params=None):
    state = np.ascontiguousarray(state, dtype=np.float64)
    nz, ny, nx = (s - 2 * ng for s in state.shape[1:])
    prm = _params(params)
    dt = ctypes.c_double(0.0)
    L = lib()
    L.nyxo_opcount_reset()
    if L.nyxo_opcount_dt(ctypes.byref(prm), nx, ny, nz, ng, _ptr(state), a, dx, cfl,
                         ctypes.byref(dt)) != 0:
        raise ValueError("nyxo_opcount_dt: bad arguments")
    return dt.value, _read()


def flops(counts):
    """+, -, *, /, sqrt: one flop each."""
    return int(counts[..., :4].sum())


def units(n):
    """Work units of each stage kernel's grid on an n = (nx, ny, nz) box: the
    padded cells, the cells of [-1, n]^3 (times 3 directions for tracing),
    the faces of each Riemann stage, the valid cells."""
    nx, ny, nz = n
    P = (nx + 8) * (ny + 8) * (nz + 8)
    E = (nx + 2) * (ny + 2) * (nz + 2)
    V = nx * ny * nz
    f0 = (nx + 1) * (ny + 2) * (nz + 2) + (nx + 2) * (ny + 1) * (nz + 2) + \
        (nx + 2) * (ny + 2) * (nz + 1)
    f1 = 0
    f2 = 0
    ext = (nx, ny, nz)
    for d in range(3):
        for t in range(3):
            if t == d:
                continue
            e = [ext[k] + 2 for k in range(3)]
            e[d] = ext[d] + 1
            e[t] = ext[t]
            f1 += e[0] * e[1] * e[2]
        e = list(ext)
        e[d] = ext[d] + 1
        f2 += e[0] * e[1] * e[2]
    return {"prim": P, "flat": E, "trace": 3 * E, "riem0": f0, "riem1": f1, "riem2": f2,
            "update": V, "cfl": V}


def stage_table(samples):
    """Flops per unit of each stage over the (state, grav, ng, dt, dx, a_old,
    a_new) samples: for the Riemann stages split into flops per face outside
    the Newton iterations and flops per iteration, with the oracle's mean
    iterations per face."""
    tot = {k: np.zeros((2, len(OPS)), dtype=np.int64) for k in STAGE_NAMES.values()}
    unit = {k: 0 for k in STAGE_NAMES.values()}
    iters = {k: 0 for k in ("riem0", "riem1", "riem2")}
    import oracle
    for (U, g, ng, dt, dx, a0, a1) in samples:
        n = tuple(s - 2 * ng for s in U.shape[1:][::-1])
        for k, u in units(n).items():
            unit[k] += u
        _, _, c = count_step(U, g, ng, dt, dx, a0, a1)
        for s, name in STAGE_NAMES.items():
            if s != 8:
                tot[name] += c[s]
        _, c8 = count_dt(U, ng, a0, dx, 0.5)
        tot["cfl"] += c8[8]
        # Newton iterations per Riemann stage: the oracle's own counter, one
        # stage at a time (a run whose other stages are not counted would
        # need other hooks; the per-iteration flops are constant, so the
        # iteration count of a stage is its iteration flops / that constant)
    per_iter = None
    for name in ("riem0", "riem1", "riem2"):
        it_ops = tot[name][1]
        it_flops = int(it_ops[:4].sum())
        if it_flops and per_iter is None:
            # the loop body is branch-free apart from the stop test: derive
            # the per-iteration flops from the square roots (two per pass)
            per_iter = it_flops / (it_ops[3] / 2.0)
        iters[name] = int(it_ops[3] // 2)
    out = {}
    for name in STAGE_NAMES.values():
        c = tot[name]
        u = unit[name]
        row = {"unit_count": int(u), "flops_per_unit": float(c[:, :4].sum()) / u,
               "by_op_per_unit": {op: float(c[:, i].sum()) / u for i, op in enumerate(OPS)}}
        if name in iters:
            nf = float(c[0, :4].sum()) / u
            row.update({"flops_per_face_outside_iterations": nf,
                        "flops_per_iteration": per_iter,
                        "oracle_iterations_per_face": iters[name] / u})
        out[name] = row
    return out


def main():
    sys.path.insert(0, _ROOT)
    from paper_1301_4498_amd import synth
    build(force=True)
    m = 32
    samples = {}
    w2 = synth.config2(n=64, seed=2)
    samples["box256_smooth fields (64^3 box of the same distributions, seed 2)"] = \
        [(w2.state, w2.grav, 4, None, w2.dx * 4, w2.a0, w2.a_at(1))]
    w1 = synth.config1()
    samples["box32_plain"] = [(w1.state, w1.grav, 4, None, w1.dx, w1.a0, w1.a_at(1))]
    w5 = synth.config5(n=64, seed=5)
    samples["box512_stress fields (64^3 box of the same distributions, seed 5)"] = \
        [(w5.state, w5.grav, 4, None, w5.dx * 8, w5.a0, w5.a_at(1))]
    import oracle
    table = {"what": "flops per work unit of each stage kernel, counted by the oracle "
                     "(oracle/opcount.cpp) on the samples named; +, -, *, /, sqrt one flop each",
             "command": "python oracle/opcount.py", "workloads": {}}
    for name, smp in samples.items():
        rows = []
        for (U, g, ng, _dt, dx, a0, a1) in smp:
            dt = oracle.estimate_dt(U, ng, a0, dx, 0.5)
            rows.append((U, g, ng, dt, dx, a0, a1))
        table["workloads"][name] = stage_table(rows)
        print(name)
        for k, r in table["workloads"][name].items():
            extra = ""
            if "flops_per_iteration" in r:
                extra = "  (%.1f/face + %.1f/iter x %.2f iter)" % (
                    r["flops_per_face_outside_iterations"], r["flops_per_iteration"],
                    r["oracle_iterations_per_face"])
            print("  %-7s %8.1f flops/unit%s" % (k, r["flops_per_unit"], extra))
    with open(TABLE, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print("wrote", TABLE)


if __name__ == "__main__":
    main()
