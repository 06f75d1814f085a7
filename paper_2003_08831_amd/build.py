"""Build libesrk.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libesrk.so")
SOURCES = ["api.cpp", "batch.cpp", "tables.cpp", "rhs.hip", "relax.hip", "ns.hip", "mlp.hip"]

HIPFLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # no packed FP32 instructions (v_pk_*_f32) anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False, extra=None, out: str = LIB) -> str:
    """Compile every source (in parallel) and link out (default: the in-tree library)."""
    from concurrent.futures import ThreadPoolExecutor

    tag = str(os.getpid())
    cmds, objs = [], []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(CSRC, f"{os.path.splitext(s)[0]}.{tag}.o")
        cmd = ["hipcc", "-c"] + [f for f in HIPFLAGS if f != "-shared"] + (extra or [])
        if s.endswith(".cpp"):
            cmd += ["-x", "hip"]
        cmd += [src, "-o", obj]
        cmds.append(cmd)
        objs.append(obj)
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    try:
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            for cmd, res in zip(cmds, ex.map(
                    lambda c: subprocess.run(c, capture_output=True, text=True), cmds)):
                if verbose or res.returncode != 0:
                    print(" ".join(cmd), flush=True)
                    sys.stderr.write(res.stderr)
                if res.returncode != 0:
                    raise subprocess.CalledProcessError(res.returncode, cmd)
        cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", "-o", out + ".tmp"] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return out


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
