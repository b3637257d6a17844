"""Build of the library with its host code under AddressSanitizer and UndefinedBehaviorSanitizer,
for the CPU-only test of the host-side validation (test infrastructure; no GPU run loads it)."""
import os
import subprocess
import tempfile

from paper_1704_05528_amd.build import CSRC, SOURCES, hipcc


def build_host_sanitized(out, verbose=False):
    """The library with its host code built with AddressSanitizer and UndefinedBehaviorSanitizer
    (each -fsanitize after -Xarch_host; the device code is built as usual, without them): for
    checking the host-side validation and bookkeeping on a machine without a GPU.  Load it with the
    clang ASan runtime preloaded."""
    cc = hipcc()
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all"]
    with tempfile.TemporaryDirectory() as tmp:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tmp, src.replace(".hip", ".o"))
            cmd = [cc, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(obj)
        for src, p in procs:
            out_, _ = p.communicate()
            if p.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n" + out_.decode(errors="replace"))
        cmd = [cc, *flags, "-shared", *objs, "-o", out]
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + r.stdout.decode(errors="replace"))
    return out
