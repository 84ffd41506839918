"""The viewer process beside the mapping loop (paper Sec. III, Fig.
"CUDA_IPC"): the mapping process exports its live parameter buffer through
the C ABI's inter-process calls, and a separate viewer process maps that
buffer and renders frames of it with the allocation-free render, while the
mapping loop keeps optimising the same memory.

    python -m paper_2509_06433_amd.viewer HANDLE_FILE --num N --stride S --deg D
        --cam R0,..,R8,t0,t1,t2,fx,fy,cx,cy,W,H (--frames K | --seconds T)
        [--fps F] [--pan DEG] [--wait-event] [--dump FILE] [--ready FILE]

HANDLE_FILE (written by SharedMap): the 64-byte memory handle, the int64 byte
offset of the parameters inside the exported allocation, and, where the
driver offers inter-process events, a 64-byte event handle the mapper
records after each iteration. The viewer prints one JSON line (frames,
seconds, fps, frame-time percentiles, GPU ms per frame, the status of its
last render).

The viewer imports torch before the library so that both processes use the
same HIP runtime (torch ships its own; a memory handle is only understood by
the runtime that made it). Per frame it makes no device allocation: the
output images are allocated once, and every render's scratch is the
library's static array. Only argument marshalling and process handling
happen here; the frames are the library's kernels.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import struct
import subprocess
import sys
import tempfile
import time

import torch

from . import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def camera_arg(cam) -> str:
    c = _lib.make_camera(cam)
    vals = list(c.R) + list(c.t) + [c.fx, c.fy, c.cx, c.cy, c.width, c.height]
    return ",".join(repr(float(v)) for v in vals)


def parse_camera(text: str) -> _lib.gsr_camera:
    v = [float(x) for x in text.split(",")]
    if len(v) != 18:
        raise ValueError("--cam takes 18 numbers: R (9), t (3), fx, fy, cx, cy, W, H")
    c = _lib.gsr_camera()
    for k in range(9):
        c.R[k] = v[k]
    for k in range(3):
        c.t[k] = v[9 + k]
    c.fx, c.fy, c.cx, c.cy = v[12:16]
    c.width, c.height = int(v[16]), int(v[17])
    return c


def panned(c: _lib.gsr_camera, deg: float) -> _lib.gsr_camera:
    """The view turned by deg degrees about its own y axis: R' = Ry R, t' = Ry t."""
    th = math.radians(deg)
    cs, sn = math.cos(th), math.sin(th)
    Ry = [[cs, 0.0, sn], [0.0, 1.0, 0.0], [-sn, 0.0, cs]]
    o = _lib.gsr_camera()
    ctypes.memmove(ctypes.addressof(o), ctypes.addressof(c), ctypes.sizeof(c))
    for r in range(3):
        for k in range(3):
            o.R[r * 3 + k] = sum(Ry[r][j] * c.R[j * 3 + k] for j in range(3))
        o.t[r] = sum(Ry[r][j] * c.t[j] for j in range(3))
    return o


class SharedMap:
    """Exports params (a [P, N] CUDA float32 view with plane stride S, inside
    an allocation of at most 1 GiB) and, with with_event, an inter-process
    event the mapper records after each iteration (record()). Where the
    driver offers no inter-process events, event is None and event_error
    holds the reason: the viewer then reads the live buffer unordered."""

    def __init__(self, params, sh_degree, with_event=True):
        self.params, self.sh_degree = params, sh_degree
        self.handle, self.offset, self.alloc_bytes = _lib.gsr_ipc_export_memory(params)
        self.event, self.event_handle, self.event_error = None, b"", None
        if with_event:
            try:
                self.event, self.event_handle = _lib.gsr_ipc_event_create()
            except _lib.GsrError as e:
                self.event_error = str(e)
        self.dir = tempfile.mkdtemp(prefix="gsr_viewer_")
        self.handle_file = os.path.join(self.dir, "handle.bin")
        with open(self.handle_file, "wb") as f:
            f.write(self.handle + struct.pack("<q", self.offset) + self.event_handle)

    def record(self, stream=None):
        if self.event is not None:
            _lib.gsr_ipc_event_record(self.event, stream)

    def close(self):
        if self.event is not None:
            _lib.gsr_ipc_event_destroy(self.event)
            self.event = None


class ViewerProcess:
    """The viewer on a SharedMap as a child process: start, then wait() for
    its JSON report."""

    def __init__(self, shared: SharedMap, cam, frames=0, seconds=0.0, fps=0.0, pan_deg=0.0, wait_event=False,
                 dump=None):
        p = shared.params
        self.ready = os.path.join(shared.dir, f"ready_{time.monotonic_ns()}")
        cmd = [sys.executable, "-m", "paper_2509_06433_amd.viewer", shared.handle_file, "--num", str(p.shape[1]),
               "--stride", str(p.stride(0)), "--deg", str(shared.sh_degree), "--cam", camera_arg(cam),
               "--ready", self.ready]
        cmd += ["--frames", str(int(frames))] if frames else ["--seconds", str(float(seconds))]
        if fps:
            cmd += ["--fps", str(float(fps))]
        if pan_deg:
            cmd += ["--pan", str(float(pan_deg))]
        if wait_event:
            cmd.append("--wait-event")
        if dump:
            cmd += ["--dump", dump]
        env = dict(os.environ)
        env["PYTHONPATH"] = ROOT + (os.pathsep + env["PYTHONPATH"] if env.get("PYTHONPATH") else "")
        self.proc = subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, close_fds=True,
                                     env=env)

    def wait_ready(self, timeout=180.0):
        """Blocks until the viewer has mapped the buffer (or has exited)."""
        t0 = time.time()
        while not os.path.exists(self.ready):
            if self.proc.poll() is not None:
                raise RuntimeError("viewer exited early: " + self.proc.stdout.read() + self.proc.stderr.read())
            if time.time() - t0 > timeout:
                raise TimeoutError("viewer did not start")
            time.sleep(0.01)

    def wait(self, timeout=300.0):
        out, err = self.proc.communicate(timeout=timeout)
        line = [ln for ln in out.splitlines() if ln.startswith("{")]
        if self.proc.returncode != 0 or not line:
            raise RuntimeError(f"viewer failed ({self.proc.returncode}): {out} {err[-2000:]}")
        rep = json.loads(line[-1])
        if "error" in rep:
            raise RuntimeError(f"viewer: {rep}")
        return rep


def read_dump(path):
    """(rgb [3,H,W], depth [H,W], alpha [H,W], camera floats [16], (W, H)) of a viewer dump."""
    import numpy as np
    raw = open(path, "rb").read()
    W, H = struct.unpack("<ii", raw[-8:])
    n = 5 * W * H
    img = np.frombuffer(raw[:4 * n], np.float32).reshape(5, H, W)
    cam = np.frombuffer(raw[4 * n:4 * n + 64], np.float32)
    return img[:3], img[3], img[4], cam, (W, H)


def _fail(what, err):
    print(json.dumps({"error": what, "detail": str(err), "status": getattr(err, "status", None),
                      "hip_error": getattr(err, "hip", None)}), flush=True)
    return 1


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_2509_06433_amd.viewer")
    ap.add_argument("handle_file")
    ap.add_argument("--num", type=int, required=True)
    ap.add_argument("--stride", type=int, required=True)
    ap.add_argument("--deg", type=int, required=True)
    ap.add_argument("--cam", required=True)
    ap.add_argument("--frames", type=int, default=0)
    ap.add_argument("--seconds", type=float, default=0.0)
    ap.add_argument("--fps", type=float, default=0.0)
    ap.add_argument("--pan", type=float, default=0.0)
    ap.add_argument("--pan-period", type=int, default=240)
    ap.add_argument("--wait-event", action="store_true")
    ap.add_argument("--dump")
    ap.add_argument("--ready")
    a = ap.parse_args(argv)
    if a.num <= 0 or a.stride < a.num or not (0 <= a.deg <= 3) or (a.frames <= 0 and a.seconds <= 0):
        ap.error("need --num > 0, --stride >= --num, --deg in 0..3 and --frames or --seconds")
    base_cam = parse_camera(a.cam)
    try:
        raw = open(a.handle_file, "rb").read()
    except OSError as e:
        return _fail("cannot read the handle file", e)
    if len(raw) < 72:
        return _fail("short handle file", ValueError(len(raw)))
    mem, offset, ev_handle = raw[:64], struct.unpack("<q", raw[64:72])[0], raw[72:136]
    torch.cuda.init()
    try:
        ptr, base = _lib.gsr_ipc_open_memory(mem, offset)
    except _lib.GsrError as e:
        return _fail("gsr_ipc_open_memory", e)
    event = None
    if a.wait_event:
        if len(ev_handle) != 64:
            return _fail("no event handle", ValueError("handle file without an event"))
        try:
            event = _lib.gsr_ipc_event_open(ev_handle)
        except _lib.GsrError as e:
            return _fail("gsr_ipc_event_open", e)
    ctx = _lib.gsr_create()
    W, H = base_cam.width, base_cam.height
    out = (torch.empty(3, H, W, device="cuda"), torch.empty(H, W, device="cuda"), torch.empty(H, W, device="cuda"))
    img = (_lib.gsr_image * 1)(_lib.gsr_image(out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr()))
    g = _lib.gsr_gaussians(ptr, a.num, a.stride, a.deg)
    stream = torch.cuda.Stream()
    sptr = ctypes.c_void_p(stream.cuda_stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    L = _lib.load()
    if a.ready:
        open(a.ready, "w").close()
    frame_ms, gpu_ms, status = [], 0.0, 0
    cams = (_lib.gsr_camera * 1)()
    t0 = time.perf_counter()
    k = 0
    while True:
        if a.frames > 0 and k >= a.frames:
            break
        el = time.perf_counter() - t0
        if a.frames <= 0 and el >= a.seconds:
            break
        if a.fps > 0:
            due = k / a.fps
            if due > el:
                time.sleep(due - el)
        f0 = time.perf_counter()
        cams[0] = panned(base_cam, a.pan * math.sin(2 * math.pi * k / a.pan_period)) if a.pan else base_cam
        if event is not None:
            _lib.gsr_ipc_event_wait(event, stream)
        e0.record(stream)
        rc = L.gsr_render_noalloc(ctx, ctypes.byref(g), 1, cams, img, sptr)
        if rc != 0:
            return _fail("gsr_render_noalloc", _lib.GsrError("gsr_render_noalloc", rc, L.gsr_last_hip_error(ctx)))
        e1.record(stream)
        stream.synchronize()
        gpu_ms += e0.elapsed_time(e1)
        frame_ms.append((time.perf_counter() - f0) * 1e3)
        k += 1
    secs = time.perf_counter() - t0
    st = _lib.gsr_query_status(ctx)
    if a.dump:
        import numpy as np
        host = np.concatenate([out[0].cpu().numpy().ravel(), out[1].cpu().numpy().ravel(), out[2].cpu().numpy().ravel()])
        c = cams[0]
        with open(a.dump, "wb") as f:
            f.write(host.astype(np.float32).tobytes())
            f.write(np.asarray(list(c.R) + list(c.t) + [c.fx, c.fy, c.cx, c.cy], np.float32).tobytes())
            f.write(struct.pack("<ii", W, H))
    s = sorted(frame_ms)
    pct = (lambda q: s[min(len(s) - 1, int(q * (len(s) - 1)))] if s else 0.0)
    print(json.dumps({"frames": k, "seconds": round(secs, 4), "fps": round(k / max(secs, 1e-9), 2),
                      "frame_ms_p50": round(pct(0.5), 4), "frame_ms_p99": round(pct(0.99), 4),
                      "gpu_ms_per_frame": round(gpu_ms / k, 4) if k else 0.0, "instances": st["instances"],
                      "status": status, "width": W, "height": H}), flush=True)
    _lib.gsr_destroy(ctx)
    _lib.gsr_ipc_close_memory(base)
    return 0


if __name__ == "__main__":
    sys.exit(main())
