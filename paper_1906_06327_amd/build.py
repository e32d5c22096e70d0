"""Build the HIP library libsscn.so for gfx950 (in-tree).

Each translation unit is compiled to an object in its own hipcc process (in
parallel), then the objects are linked into the shared library."""
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
# (source, extra defines): the kernel launchers are compiled once per part
# (1 sweeps, 2, 4 and 5 the fused 2D step's three tile shapes, 3 batched
# sweeps) and precision
UNITS = [(os.path.join(CSRC, "sscn_lib.hip"), []), (os.path.join(CSRC, "sscn_nn.hip"), []),
         (os.path.join(CSRC, "sscn_setup.cpp"), [])] + [
    (os.path.join(CSRC, "sscn_kernels.hip"), [f"-DSSCN_PART={part}", f"-DSSCN_REAL_T={real}"])
    for part in (2, 4, 5, 1, 3) for real in ("double", "float")]
LIB = os.path.join(HERE, "libsscn.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions (v_pk_*_f32) stay off: some of their forms have
    # produced wrong results without any error on gfx950 parts
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast", "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
]


def build(verbose: bool = False, extra_flags=(), out: str = LIB) -> str:
    """Compile every translation unit (extra_flags appended to each hipcc
    line, e.g. -D overrides of the tuning constants) and link `out`."""
    with tempfile.TemporaryDirectory(prefix="sscn_build_") as tmp:
        objs, procs = [], []
        for n, (src, defs) in enumerate(UNITS):
            obj = os.path.join(tmp, f"{n}_{os.path.basename(src)}.o")
            cmd = [HIPCC] + FLAGS + defs + list(extra_flags) + ["-c", "-o", obj, src]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((cmd, subprocess.Popen(cmd)))
            objs.append(obj)
        codes = [pr.wait() for _, pr in procs]  # every compiler finishes before the directory goes
        for (cmd, _), rc in zip(procs, codes):
            if rc != 0:
                raise subprocess.CalledProcessError(rc, cmd)
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out + ".tmp"] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
