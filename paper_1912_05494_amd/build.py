"""Build ``libsdm.so`` (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libsdm.so")
SOURCES = ["api.cpp", "render.cpp", "bvh_build.cpp", "sun_grid.cpp", "subdomain.cpp", "wavefront.hip",
           "surrogate.hip"]
ARCH = os.environ.get("SDM_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # packed FP32 instructions are kept out of the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-result"]
# the render's surrogate evaluation keeps its matrix-core accumulators in
# ordinary VGPRs (no accumulator-register reads between the layers)
SOURCE_FLAGS = {"wavefront.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def build(verbose=False, jobs=None):
    objs = []
    with tempfile.TemporaryDirectory() as td:
        procs = []
        for src in SOURCES:
            obj = os.path.join(td, os.path.basename(src) + ".o")
            cmd = ["hipcc", "-x", "hip", *FLAGS, *SOURCE_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), file=sys.stderr)
            procs.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), src))
            objs.append(obj)
        failed = []
        for p, src in procs:
            out, _ = p.communicate()
            text = out.decode(errors="replace")
            if p.returncode != 0:
                failed.append((src, text))
            elif verbose and text.strip():
                print(text, file=sys.stderr)
        if failed:
            for src, text in failed:
                print(f"--- {src}\n{text}", file=sys.stderr)
            raise RuntimeError("hipcc failed for " + ", ".join(s for s, _ in failed))
        cmd = ["hipcc", *FLAGS, "-shared", "-o", SO + ".tmp", *objs]
        subprocess.run(cmd, check=True)
    os.replace(SO + ".tmp", SO)
    return SO


def ensure_built():
    """Build only when no library is present."""
    if not os.path.exists(SO):
        build()
    return SO


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
