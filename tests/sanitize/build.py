"""Build of the sanitizer driver (test infrastructure): the library's host code
compiled for the host only, linked against the fake HIP device instead of the
HIP runtime, with AddressSanitizer + UndefinedBehaviorSanitizer or with
ThreadSanitizer.  The kernels' host stubs are compiled, their device code is
not (a kernel "runs" on the fake device by checking the memory it would touch).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2507_01522_amd", "csrc")
INC = os.path.join(ROOT, "include")
CLANGXX = "/opt/rocm/llvm/bin/clang++"

LIB_SOURCES = ["cx_kernels.hip", "cx_policy.hip", "cx_api.cpp", "cx_spec.cpp", "cx_state.cpp", "cx_tune.cpp",
               "cx_server.cpp"]

SANITIZERS = {
    "asan": ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-fno-sanitize-recover=undefined"],
    "tsan": ["-Xarch_host", "-fsanitize=thread"],
}
LINK = {"asan": ["-fsanitize=address", "-fsanitize=undefined"], "tsan": ["-fsanitize=thread"]}


def _compile(src: str, out_dir: str, kind: str) -> str:
    path = src if os.path.isabs(src) else os.path.join(CSRC, src)
    obj = os.path.join(out_dir, os.path.basename(path) + ".o")
    cmd = ["hipcc", "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer", f"-I{INC}", f"-I{CSRC}",
           "-DCX_AUTOTUNE_ON=1", "-Wno-unused-command-line-argument", *SANITIZERS[kind]]
    base = os.path.basename(path)
    # every file as HIP (as the library's build compiles them), host side only
    cmd += ["-x", "hip", "--offload-host-only"]
    if base == "cx_spec.cpp":
        cmd += ["-ffp-contract=off"]
    cmd += ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {base} ({kind}) failed:\n{r.stderr}")
    return obj


def build(kind: str, out_dir: str) -> str:
    """Compile and link the driver for one sanitizer; returns the executable."""
    os.makedirs(out_dir, exist_ok=True)
    srcs = LIB_SOURCES + [os.path.join(HERE, "fake_hip.cpp"), os.path.join(HERE, "drive.cpp")]
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, out_dir, kind), srcs))
    # the device-code blobs the host objects refer to (there is no device code):
    # defined empty, so the objects link without the HIP runtime
    names = set()
    for o in objs:
        r = subprocess.run(["nm", "-u", o], capture_output=True, text=True, check=True)
        names |= {ln.split()[-1] for ln in r.stdout.splitlines() if "__hip_fatbin_" in ln}
    blobs = os.path.abspath(os.path.join(out_dir, "fatbin_blobs.cpp"))
    with open(blobs, "w") as f:
        f.write("".join(f'extern "C" {{ char {n}[16]; }}\n' for n in sorted(names)))
    objs.append(_compile(blobs, out_dir, kind))
    exe = os.path.join(out_dir, f"drive_{kind}")
    r = subprocess.run([CLANGXX, *LINK[kind], "-o", exe, *objs, "-lpthread"], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link ({kind}) failed:\n{r.stderr}")
    return exe


def write_scenario(path: str) -> None:
    """Station specs of the driver's scenario: the uneven mixture's 15 classes
    plus a general, a V2G / battery and a table-driven class, with ragged env
    counts; the policy station; a few served classes."""
    import numpy as np

    import workloads as W
    mix = W.mixture_classes() + [W.two_charger_types(), W.v2g_station(),
                                 W.exo_station(), W.user_station()]
    counts = [40, 30, 20, 30, 25, 20, 15, 12, 10, 9, 8, 7, 3, 2, 2, 11, 9, 13, 6]
    served = W.mixture_classes()[::4] + [W.v2g_station(), W.exo_station()]

    def spec_lines(s):
        out = ["spec"]
        for f in ("n_ports", "node_parent", "node_limit_kw", "node_eta", "port_parent", "port_pmax_kw", "port_eta",
                  "dt_hours", "tau", "p_sell", "p_sell_grid", "fixed_cost", "alpha_sat", "alpha_declined",
                  "steps_per_episode", "n_levels", "price_base", "price_amp", "price_sigma", "arrival_peak",
                  "cap_lo", "cap_hi", "soc0_lo", "soc0_hi", "tgt_lo", "tgt_hi", "dwell_mu", "dwell_sigma",
                  "dwell_max", "arrival_rate", "price_table", "v2g", "port_pdis_kw", "battery_kwh", "battery_kw",
                  "battery_tau", "battery_soc0", "alpha_degrad_battery", "alpha_degrad_cars",
                  "charge_sensitive_share", "alpha_sat1", "beta_sat1", "price_days", "car_models", "port_dc"):
            v = getattr(s, f, None)
            if v is None:
                continue
            vals = np.asarray(v, dtype=np.float64).ravel()
            out.append(f + " " + " ".join(repr(float(x)) for x in vals))
        out.append("end")
        return out

    lines = ["section mixture", "counts " + " ".join(str(c) for c in counts)]
    for s in mix:
        lines += spec_lines(s)
    lines.append("section policy")
    lines += spec_lines(W.policy_station())
    lines.append("section serve")
    for s in served:
        lines += spec_lines(s)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")

