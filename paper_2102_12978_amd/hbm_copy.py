"""Plain device-to-device copy of a known size, used to calibrate the HBM
byte counters (FETCH_SIZE, WRITE_SIZE) read by rocprofv3 --pmc, and the
library's streaming probe (fdtd_stream_probe): the bandwidth a kernel with
no arithmetic reaches for a copy, a read-only and a write-only pass.

    python -m paper_2102_12978_amd.hbm_copy [--mib 1024] [--reps 5]
    python -m paper_2102_12978_amd.hbm_copy --probe [--mib 2048] [--reps 20]
"""
import argparse
import ctypes

from . import _lib as L

PROBE_COPY, PROBE_READ, PROBE_WRITE = 0, 1, 2


def stream_probe(kind, nbytes, reps=20, stream=None):
    """(ms per pass, GB/s) of the library's streaming kernel of `kind`."""
    lib = L.load()
    ms = ctypes.c_double()
    gbs = ctypes.c_double()
    rc = lib.fdtd_stream_probe(int(kind), int(nbytes), int(reps), stream, ctypes.byref(ms),
                               ctypes.byref(gbs))
    if rc != 0:
        raise L.FdtdError(rc, "fdtd_stream_probe failed")
    return ms.value, gbs.value


def stream_ceiling(nbytes=1 << 31, reps=20, stream=None):
    """Copy, read-only and write-only GB/s over buffers of nbytes (2 GiB by
    default: eight times the 256 MB last-level cache)."""
    return {"bytes": int(nbytes),
            "copy_gbs": round(stream_probe(PROBE_COPY, nbytes, reps, stream)[1], 1),
            "read_gbs": round(stream_probe(PROBE_READ, nbytes, reps, stream)[1], 1),
            "write_gbs": round(stream_probe(PROBE_WRITE, nbytes, reps, stream)[1], 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--probe", action="store_true", help="run the library's streaming probe")
    a = ap.parse_args()
    if a.probe:
        print(stream_ceiling(a.mib * (1 << 20), a.reps))
        return
    import torch
    n = a.mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {a.mib} MiB x {a.reps}: {a.mib * (1 << 20)} bytes read and written per copy")


if __name__ == "__main__":
    main()
