"""Thin ctypes binding of libart.so (argument marshalling only).

Every step of the render runs in the HIP kernels behind the C ABI declared in
include/art.h; this module builds the parameter blocks, allocates the output
tensors with PyTorch on the current CUDA (HIP) device and passes raw pointers
and the current stream.  There is no CPU fallback: if the library is missing
or no GPU is present, calls raise.
"""
import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libart.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "art.h")

EMIS = {"toy_disk": 1, "thermal": 2, "grid": 3, "screen_ring": 10, "screen_poly": 11}
NORM = {"mean": 0, "max": 1}
INTERP = {"linear": 0, "nearest": 1}
PREC = {"fp64": 0, "mixed": 1, "mixed_geo": 2}
STATUS_NAMES = ("ok", "captured", "escaped", "step_cap", "thick", "nan")


class ArtError(RuntimeError):
    pass


class Spacetime(ctypes.Structure):
    _fields_ = [("a_spin", ctypes.c_double)]


class Camera(ctypes.Structure):
    _fields_ = [("r_cam", ctypes.c_double), ("inc_deg", ctypes.c_double),
                ("fov_M", ctypes.c_double), ("r_out", ctypes.c_double),
                ("nx0", ctypes.c_int32), ("ny0", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("pad", ctypes.c_int32), ("phi_deg", ctypes.c_double)]


class Emission(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("freq_hz", ctypes.c_double), ("mass_msun", ctypes.c_double),
                ("params", ctypes.c_double * 16),
                ("grid_dev", ctypes.c_void_p), ("grid_len", ctypes.c_int64)]


class Refine(ctypes.Structure):
    _fields_ = [("r_rel", ctypes.c_double), ("r_abs", ctypes.c_double),
                ("abs_norm", ctypes.c_int32), ("interp", ctypes.c_int32),
                ("all_planes", ctypes.c_int32), ("pad", ctypes.c_int32)]


class Transfer(ctypes.Structure):
    _fields_ = [("nstokes", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("max_steps", ctypes.c_int32), ("subrings", ctypes.c_int32),
                ("eps", ctypes.c_double), ("fp64_radius", ctypes.c_double),
                ("fp64_ktheta", ctypes.c_double)]


class Image(ctypes.Structure):
    _fields_ = [("image_dev", ctypes.c_void_p), ("level_dev", ctypes.c_void_p),
                ("feat_dev", ctypes.c_void_p), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("rays_traced", ctypes.c_int64), ("candidates", ctypes.c_int64 * 32),
                ("traced", ctypes.c_int64 * 32), ("steps_total", ctypes.c_int64),
                ("status_hist", ctypes.c_int64 * 8), ("interp_frac", ctypes.c_double),
                ("ibar_int", ctypes.c_double), ("imax0", ctypes.c_double),
                ("n_abs", ctypes.c_double), ("steps_emit", ctypes.c_int64),
                ("t_trace_ms", ctypes.c_double), ("trace_launches", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("learned", ctypes.c_int64 * 5),
                ("t_render_ms", ctypes.c_double), ("spectral", ctypes.c_int64)]


class Spectral(ctypes.Structure):
    _fields_ = [("nu_min_hz", ctypes.c_double), ("nu_max_hz", ctypes.c_double),
                ("n0", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("r_rel", ctypes.c_double), ("r_abs", ctypes.c_double)]


class Learned(ctypes.Structure):
    _fields_ = [("z_propose", ctypes.c_float), ("z_suppress", ctypes.c_float),
                ("fallback", ctypes.c_int32), ("all_levels", ctypes.c_int32),
                ("level_cap", ctypes.c_int32), ("pad", ctypes.c_int32)]


class Job(ctypes.Structure):
    _fields_ = [("sp", Spacetime), ("cam", Camera), ("em", Emission), ("rf", Refine),
                ("tr", Transfer)]


class Launch(ctypes.Structure):
    _fields_ = [("trace_blocks", ctypes.c_int32), ("trace_threads", ctypes.c_int32),
                ("refill", ctypes.c_int32), ("groups", ctypes.c_int32),
                ("refine_blocks", ctypes.c_int32), ("long_steps", ctypes.c_int32)]


FEAT_DTYPE = np.dtype([("rmin", np.float32), ("ncross", np.int32),
                       ("steps", np.int32), ("status", np.int32)])

_lib = None


def header_functions():
    """Names of the functions declared in include/art.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char\*)\s+(art_\w+)\s*\(", txt, re.M)))


def lib():
    """Load libart.so (raises ArtError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ArtError("libart.so not found at %s: run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        P = ctypes.POINTER
        L.art_image_size.argtypes = [P(Camera), ctypes.c_int32, P(ctypes.c_int32),
                                     P(ctypes.c_int32), P(ctypes.c_size_t)]
        L.art_render.argtypes = [P(Spacetime), P(Camera), P(Emission), P(Refine), P(Transfer),
                                 P(Image), P(Stats), vp]
        L.art_render_noalloc.argtypes = [P(Spacetime), P(Camera), P(Emission), P(Refine), P(Transfer),
                                         P(Image), P(Stats), vp]
        L.art_set_alloc_limit.argtypes = [ctypes.c_size_t]
        L.art_render_uniform.argtypes = [P(Spacetime), P(Camera), P(Emission), P(Transfer),
                                         P(Image), P(Stats), vp]
        L.art_trace_points.argtypes = [P(Spacetime), P(Camera), P(Emission), P(Transfer), i64,
                                       vp, vp, vp, vp, vp]
        L.art_metrics.argtypes = [vp, vp, i64, P(ctypes.c_double), P(ctypes.c_double), vp]
        L.art_batch_create.argtypes = [ctypes.c_int32, P(Job), P(Image), P(vp)]
        L.art_cube_create.argtypes = [ctypes.c_int32, P(Job), ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                      ctypes.c_double, P(Image), P(vp)]
        L.art_batch_render.argtypes = [vp, vp]
        L.art_batch_capture.argtypes = [vp, vp]
        L.art_batch_launch.argtypes = [vp, vp]
        L.art_batch_stats.argtypes = [vp, ctypes.c_int32, P(Stats), vp]
        L.art_batch_destroy.argtypes = [vp]
        L.art_set_launch.argtypes = [P(Launch)]
        L.art_batch_set_launch.argtypes = [vp, P(Launch)]
        L.art_batch_get_launch.argtypes = [vp, P(Launch)]
        L.art_get_launch.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P(Launch)]
        f32, u64, i32 = ctypes.c_float, ctypes.c_uint64, ctypes.c_int32
        L.art_cnn_num_params.argtypes = []
        L.art_cnn_create.argtypes = [u64, P(vp)]
        L.art_cnn_destroy.argtypes = [vp]
        L.art_cnn_set_params.argtypes = [vp, vp, i64]
        L.art_cnn_get_params.argtypes = [vp, vp, i64]
        L.art_cnn_forward.argtypes = [vp, vp, i32, i32, i32, vp, vp]
        L.art_cnn_gradients.argtypes = [vp, vp, vp, vp, i32, i32, i32, f32, vp, P(f32), vp]
        L.art_cnn_train_step.argtypes = [vp, vp, vp, vp, i32, i32, i32, f32, f32, P(f32), vp]
        L.art_cnn_features.argtypes = [vp, vp, i32, i32, i32, i32, i32, i32, ctypes.c_double, vp, vp]
        L.art_cnn_labels.argtypes = [vp, i32, i32, i32, i32, i32, i32, vp, vp, vp]
        L.art_batch_set_learned.argtypes = [vp, vp, P(Learned)]
        L.art_render_learned.argtypes = [P(Spacetime), P(Camera), P(Emission), P(Refine),
                                         P(Transfer), vp, P(Learned), P(Image), P(Stats), vp]
        L.art_render_spectral.argtypes = [P(Spacetime), P(Camera), P(Emission), P(Refine), P(Transfer),
                                          P(Spectral), P(Image), P(Stats), vp]
        L.art_render_cube.argtypes = [i32, P(Job), i32, i32, ctypes.c_double, ctypes.c_double, P(Image),
                                      P(Stats), vp]
        L.art_vis_workspace_bytes.argtypes = [i32, i32, i32, i32, i32]
        L.art_vis_workspace_bytes.restype = ctypes.c_size_t
        L.art_visibility.argtypes = [vp, i64, i32, i32, i32, ctypes.c_double, ctypes.c_double, vp, i32,
                                     vp, i32, vp, vp, ctypes.c_size_t, vp]
        L.art_stream_create.argtypes = [P(vp)]
        L.art_stream_destroy.argtypes = [vp]
        L.art_last_error.restype = ctypes.c_char_p
        L.art_last_error.argtypes = []
        L.art_release.argtypes = []
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        msg = lib().art_last_error().decode()
        raise ArtError("art error %d: %s" % (rc, msg))


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise ArtError("no GPU available: the HIP path has no CPU fallback")
    return torch


def blocks(cfg):
    """C parameter blocks from a workload dictionary."""
    sp = Spacetime(float(cfg["a"]))
    cam = Camera(float(cfg["r_cam"]), float(cfg["inc_deg"]), float(cfg["fov"]),
                 float(cfg.get("r_out", cfg["r_cam"])), int(cfg.get("nx0", 2)),
                 int(cfg.get("ny0", cfg.get("nx0", 2))), int(cfg.get("levels", 0)), 0,
                 float(cfg.get("phi_deg", 0.0)))
    em = Emission()
    em.kind = EMIS[cfg["model"]]
    em.freq_hz = float(cfg.get("freq_hz", 230e9))
    em.mass_msun = float(cfg.get("mass_msun", 4.0e6))
    mp = list(cfg.get("mp", []))
    for i in range(16):
        em.params[i] = float(mp[i]) if i < len(mp) else 0.0
    g = cfg.get("grid_dev")
    if g is not None:
        em.grid_dev = g.data_ptr()
        em.grid_len = g.numel()
    rf = Refine(float(cfg.get("r_rel", -1.0)), float(cfg.get("r_abs", -1.0)),
                NORM[cfg.get("abs_norm", "mean")], INTERP[cfg.get("interp", "linear")],
                2 if cfg.get("all_planes", False) == "own" else (1 if cfg.get("all_planes", False) else 0), 0)
    tr = Transfer(int(cfg.get("nstokes", 1)), PREC[cfg.get("precision", "fp64")],
                  int(cfg.get("max_steps", 100000)), int(cfg.get("subrings", 0)), float(cfg.get("eps", 0.03)),
                  float(cfg.get("fp64_radius", 0.0)), float(cfg.get("fp64_ktheta", -1.0)))
    return sp, cam, em, rf, tr


def image_size(cfg):
    _, cam, _, _, tr = blocks(cfg)
    nx, ny, nb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
    _check(lib().art_image_size(ctypes.byref(cam), tr.nstokes, ctypes.byref(nx), ctypes.byref(ny),
                                ctypes.byref(nb)))
    return nx.value, ny.value


def _stream(torch, stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def stats_dict(st):
    L = st.levels
    return dict(rays=int(st.rays_traced), traced=[int(st.traced[i]) for i in range(L + 1)],
                candidates=[int(st.candidates[i]) for i in range(L + 1)],
                steps=int(st.steps_total),
                status={STATUS_NAMES[k]: int(st.status_hist[k]) for k in range(6)},
                interp_frac=float(st.interp_frac), ibar=float(st.ibar_int),
                imax0=float(st.imax0), n_abs=float(st.n_abs), levels=L,
                steps_emit=int(st.steps_emit), t_trace_ms=float(st.t_trace_ms),
                trace_launches=int(st.trace_launches),
                learned=dict(proposed_extra=int(st.learned[0]), suppressed=int(st.learned[1]),
                             fallback=int(st.learned[2]), missed=int(st.learned[3]),
                             lookahead=int(st.learned[4])),
                t_render_ms=float(st.t_render_ms), spectral=int(st.spectral))


def alloc(cfg, feat=False):
    """Output tensors for a render of cfg: image (nstokes + subrings, ny, nx)
    float64, level map (ny, nx) int8, optional features (ny, nx, 4) int32 view."""
    torch = _torch()
    nx, ny = image_size(cfg)
    ns = int(cfg.get("nstokes", 1)) + int(cfg.get("subrings", 0))
    img = torch.empty((ns, ny, nx), dtype=torch.float64, device="cuda")
    lev = torch.empty((ny, nx), dtype=torch.int8, device="cuda")
    ft = torch.empty((ny, nx, 4), dtype=torch.int32, device="cuda") if feat else None
    return img, lev, ft


def _image(img, lev, ft):
    ny, nx = img.shape[1], img.shape[2]
    return Image(img.data_ptr(), lev.data_ptr() if lev is not None else None,
                 ft.data_ptr() if ft is not None else None, nx, ny)


def render(cfg, out=None, feat=False, stats=True, stream=None):
    """Adaptive render (Sec. 3.2).  Returns (image, level, feat, stats)."""
    torch = _torch()
    sp, cam, em, rf, tr = blocks(cfg)
    img, lev, ft = out if out is not None else alloc(cfg, feat)
    im = _image(img, lev, ft)
    st = Stats()
    rc = lib().art_render(ctypes.byref(sp), ctypes.byref(cam), ctypes.byref(em), ctypes.byref(rf),
                          ctypes.byref(tr), ctypes.byref(im),
                          ctypes.byref(st) if stats else None, _stream(torch, stream))
    _check(rc)
    return img, lev, ft, (stats_dict(st) if stats else None)


def set_alloc_limit(nbytes):
    """Bound the trace-list + cost-map allocation of later renders and batch
    set-ups (bytes; 0 = no bound)."""
    _check(lib().art_set_alloc_limit(int(nbytes)))


def render_noalloc(cfg, out, stats=True, stream=None):
    """Adaptive render through the entry point that allocates nothing (the
    library's static scratch; images up to 2049^2).  `out` = (image, level,
    feat or None), caller-allocated.  Returns (image, level, feat, stats)."""
    torch = _torch()
    sp, cam, em, rf, tr = blocks(cfg)
    img, lev, ft = out
    im = _image(img, lev, ft)
    st = Stats()
    rc = lib().art_render_noalloc(ctypes.byref(sp), ctypes.byref(cam), ctypes.byref(em), ctypes.byref(rf),
                                  ctypes.byref(tr), ctypes.byref(im),
                                  ctypes.byref(st) if stats else None, _stream(torch, stream))
    _check(rc)
    return img, lev, ft, (stats_dict(st) if stats else None)


def render_uniform(cfg, out=None, feat=False, stats=True, stream=None):
    """One ray per vertex of the final grid.  Returns (image, feat, stats)."""
    torch = _torch()
    sp, cam, em, rf, tr = blocks(cfg)
    img, lev, ft = out if out is not None else alloc(cfg, feat)
    im = _image(img, lev, ft)
    st = Stats()
    rc = lib().art_render_uniform(ctypes.byref(sp), ctypes.byref(cam), ctypes.byref(em),
                                  ctypes.byref(tr), ctypes.byref(im),
                                  ctypes.byref(st) if stats else None, _stream(torch, stream))
    _check(rc)
    return img, ft, (stats_dict(st) if stats else None)


def cube_size(n0, levels):
    return (1 << int(levels)) * (int(n0) - 1) + 1


def render_spectral(cfg, nu_min, nu_max, n0, levels, r_rel=None, r_abs=None, feat=False, stream=None):
    """Spectral cube by adaptive sampling along ln nu (the frequency-domain
    extension of Sec. 3.2 proposed in Sec. 6).  Returns (images, levels,
    feats, stats), lists in frequency order; r_rel / r_abs default to the
    spatial tolerances."""
    torch = _torch()
    sp, cam, em, rf, tr = blocks(cfg)
    n = cube_size(n0, levels)
    bufs = [alloc(cfg, feat) for _ in range(n)]
    ims = (Image * n)(*[_image(*b) for b in bufs])
    sts = (Stats * n)()
    spec = Spectral(float(nu_min), float(nu_max), int(n0), int(levels),
                    float(cfg["r_rel"] if r_rel is None else r_rel),
                    float(cfg["r_abs"] if r_abs is None else r_abs))
    rc = lib().art_render_spectral(ctypes.byref(sp), ctypes.byref(cam), ctypes.byref(em), ctypes.byref(rf),
                                   ctypes.byref(tr), ctypes.byref(spec), ims, sts, _stream(torch, stream))
    _check(rc)
    out = [stats_dict(sts[i]) for i in range(n)]
    return [b[0] for b in bufs], [b[1] for b in bufs], [b[2] for b in bufs], out


def render_cube(cfgs, n0, levels, r_rel=None, r_abs=None, feat=False, stream=None):
    """Adaptive sampling along a sequence axis (time, frequency, ...): cfgs in
    axis order, equally spaced along it, len(cfgs) = 2^levels (n0 - 1) + 1.
    Returns (images, levels, feats, stats) in axis order; r_rel / r_abs
    default to the spatial tolerances of cfgs[0]."""
    torch = _torch()
    n = len(cfgs)
    jobs = (Job * n)()
    bufs = []
    for i, c in enumerate(cfgs):
        sp, cam, em, rf, tr = blocks(c)
        jobs[i] = Job(sp, cam, em, rf, tr)
        bufs.append(alloc(c, feat))
    ims = (Image * n)(*[_image(*b) for b in bufs])
    sts = (Stats * n)()
    rc = lib().art_render_cube(n, jobs, int(n0), int(levels),
                               float(cfgs[0]["r_rel"] if r_rel is None else r_rel),
                               float(cfgs[0]["r_abs"] if r_abs is None else r_abs),
                               ims, sts, _stream(torch, stream))
    _check(rc)
    return [b[0] for b in bufs], [b[1] for b in bufs], [b[2] for b in bufs], \
        [stats_dict(sts[i]) for i in range(n)]


def learned_opts(z_propose=2.0, z_suppress=float("-inf"), fallback=True, all_levels=False, level_cap=0):
    return Learned(float(z_propose), float(z_suppress), 1 if fallback else 0, 1 if all_levels else 0,
                   int(level_cap), 0)


def render_learned(cfg, net, out=None, stats=True, stream=None, **opts):
    """Learned adaptive render (network look-ahead, criterion as judge and
    fallback).  Returns (image, level, feat, stats)."""
    torch = _torch()
    sp, cam, em, rf, tr = blocks(cfg)
    img, lev, ft = out if out is not None else alloc(cfg, True)
    im = _image(img, lev, ft)
    st = Stats()
    lo = learned_opts(**opts)
    rc = lib().art_render_learned(ctypes.byref(sp), ctypes.byref(cam), ctypes.byref(em),
                                  ctypes.byref(rf), ctypes.byref(tr), net.handle, ctypes.byref(lo),
                                  ctypes.byref(im), ctypes.byref(st) if stats else None,
                                  _stream(torch, stream))
    _check(rc)
    return img, lev, ft, (stats_dict(st) if stats else None)


def trace_points(cfg, alpha, beta, feat=True, stream=None):
    """Trace arbitrary screen points.  alpha, beta: CUDA float64 tensors.
    Returns (stokes (n, nstokes + subrings) float64, feat (n, 4) int32 or None)."""
    torch = _torch()
    sp, cam, em, rf, tr = blocks(cfg)
    alpha = alpha.contiguous()
    beta = beta.contiguous()
    n = alpha.numel()
    S = torch.empty((n, tr.nstokes + tr.subrings), dtype=torch.float64, device=alpha.device)
    ft = torch.empty((n, 4), dtype=torch.int32, device=alpha.device) if feat else None
    rc = lib().art_trace_points(ctypes.byref(sp), ctypes.byref(cam), ctypes.byref(em),
                                ctypes.byref(tr), n, alpha.data_ptr(), beta.data_ptr(),
                                S.data_ptr(), ft.data_ptr() if ft is not None else None,
                                _stream(torch, stream))
    _check(rc)
    return S, ft


def metrics(truth, approx, stream=None):
    """(flux error, normalised MSE) of two same-shape FP64 CUDA tensors (Eqs. 8-9)."""
    torch = _torch()
    t = truth.contiguous()
    a = approx.contiguous()
    fe, mse = ctypes.c_double(), ctypes.c_double()
    _check(lib().art_metrics(t.data_ptr(), a.data_ptr(), t.numel(), ctypes.byref(fe),
                             ctypes.byref(mse), _stream(torch, stream)))
    return fe.value, mse.value


def visibility(img, dx, u, v, fwhm=0.0, stream=None):
    """Visibilities V[..., l, m] = V(u_m, v_l) (complex128, device) of FP64
    image planes img[..., ny, nx] (Sec. 4.3; u, v in cycles per unit of
    screen coordinate, pixel size dx, Gaussian taper FWHM fwhm, <= 0: none)."""
    torch = _torch()
    if img.dtype != torch.float64 or not img.is_cuda:
        raise ArtError("visibility: the image must be a float64 CUDA tensor")
    if img.dim() < 2:
        raise ArtError("visibility: the image needs at least two dimensions (ny, nx)")
    cur = torch.cuda.current_stream(img.device)
    st = stream if stream is not None else cur
    x = img.contiguous()
    ny, nx = x.shape[-2], x.shape[-1]
    lead = tuple(x.shape[:-2])
    P = 1
    for d in lead:
        P *= d
    uu = torch.as_tensor(u, dtype=torch.float64).reshape(-1).to(x.device).contiguous()
    vv = torch.as_tensor(v, dtype=torch.float64).reshape(-1).to(x.device).contiguous()
    nu, nv = uu.numel(), vv.numel()
    out = torch.empty(lead + (nv, nu, 2), dtype=torch.float64, device=x.device)
    nbytes = lib().art_vis_workspace_bytes(P, nx, ny, nu, nv)
    work = torch.empty(max(nbytes // 8, 1), dtype=torch.float64, device=x.device)
    if st != cur:
        st.wait_stream(cur)
        for t in (x, uu, vv, out, work):
            t.record_stream(st)
    _check(lib().art_visibility(x.data_ptr() if x.numel() else None, ny * nx, P, nx, ny, float(dx),
                                float(fwhm), uu.data_ptr(), nu, vv.data_ptr(), nv,
                                out.data_ptr(), work.data_ptr(), nbytes, ctypes.c_void_p(st.cuda_stream)))
    return torch.view_as_complex(out)


class Stream:
    """A library-created non-blocking HIP stream (art_stream_create) as a
    torch stream (`.torch`); batches replayed on distinct such streams run
    concurrently."""

    def __init__(self):
        torch = _torch()
        h = ctypes.c_void_p()
        _check(lib().art_stream_create(ctypes.byref(h)))
        self._h = h
        self.torch = torch.cuda.ExternalStream(h.value)

    def close(self):
        if self._h:
            _check(lib().art_stream_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def feat_numpy(ft):
    """Structured numpy view (rmin, ncross, steps, status) of a feature tensor."""
    a = ft.cpu().contiguous().numpy()
    return a.view(FEAT_DTYPE).reshape(a.shape[:-1])


def set_launch(trace_blocks=0, trace_threads=0, refill=0, groups=0, refine_blocks=0, long_steps=0):
    """Persistent-tracer launch shape for later renders (0 = default)."""
    _check(lib().art_set_launch(ctypes.byref(Launch(trace_blocks, trace_threads, refill, groups,
                                                    refine_blocks, long_steps))))


def get_launch(cfg):
    _, _, em, _, tr = blocks(cfg)
    L = Launch()
    _check(lib().art_get_launch(tr.precision, em.kind, tr.nstokes, ctypes.byref(L)))
    return dict(trace_blocks=L.trace_blocks, trace_threads=L.trace_threads, refill=L.refill,
                groups=L.groups, refine_blocks=L.refine_blocks, long_steps=L.long_steps)


class Batch:
    """Many adaptive images rendered together (one work queue per level).

    cfgs: list of workload dictionaries (same model, nstokes, precision).
    Outputs are allocated here: self.images[i] (nstokes, ny, nx) float64,
    self.levels[i] (ny, nx) int8, self.feats[i] or None.
    """

    def __init__(self, cfgs, feat=False, cube=None):
        """cube=(n0, levels, r_rel, r_abs): the images form an axis-sampled
        cube (cfgs in axis order, see render_cube) rendered as one batch."""
        self._torch = _torch()
        n = len(cfgs)
        self.cfgs = list(cfgs)
        jobs = (Job * n)()
        ims = (Image * n)()
        self.images, self.levels, self.feats = [], [], []
        for i, c in enumerate(cfgs):
            sp, cam, em, rf, tr = blocks(c)
            jobs[i] = Job(sp, cam, em, rf, tr)
            img, lev, ft = alloc(c, feat)
            self.images.append(img)
            self.levels.append(lev)
            self.feats.append(ft)
            ims[i] = _image(img, lev, ft)
        self._torch.cuda.synchronize()
        h = ctypes.c_void_p()
        if cube is None:
            _check(lib().art_batch_create(n, jobs, ims, ctypes.byref(h)))
        else:
            n0, lv, rr, ra = cube
            _check(lib().art_cube_create(n, jobs, int(n0), int(lv), float(rr), float(ra), ims, ctypes.byref(h)))
        self._h = h

    def render(self, stream=None):
        _check(lib().art_batch_render(self._h, _stream(self._torch, stream)))

    def capture(self, stream):
        """Capture the level loop into a hipGraph (stream must not be the default)."""
        _check(lib().art_batch_capture(self._h, ctypes.c_void_p(stream.cuda_stream)))

    def launch(self, stream):
        _check(lib().art_batch_launch(self._h, ctypes.c_void_p(stream.cuda_stream)))

    def stats(self, i=-1, stream=None):
        st = Stats()
        _check(lib().art_batch_stats(self._h, int(i), ctypes.byref(st), _stream(self._torch, stream)))
        return stats_dict(st)

    def set_launch(self, trace_blocks=0, trace_threads=0, refill=0, groups=0, refine_blocks=0, long_steps=0):
        _check(lib().art_batch_set_launch(self._h, ctypes.byref(Launch(trace_blocks, trace_threads,
                                                                         refill, groups, refine_blocks,
                                                                         long_steps))))

    def get_launch(self):
        L = Launch()
        _check(lib().art_batch_get_launch(self._h, ctypes.byref(L)))
        return dict(trace_blocks=L.trace_blocks, trace_threads=L.trace_threads, refill=L.refill,
                    groups=L.groups, refine_blocks=L.refine_blocks, long_steps=L.long_steps)

    def set_learned(self, net, **opts):
        """Use the network `net` (a Cnn, or None for plain renders) in later
        renders and captures of this batch."""
        lo = learned_opts(**opts)
        self._net = net                      # keep the network alive while used
        _check(lib().art_batch_set_learned(self._h, net.handle if net is not None else None,
                                           ctypes.byref(lo)))

    def close(self):
        if getattr(self, "_h", None):
            lib().art_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Cnn:
    """Learned refinement proposal network (BF16 MFMA forward and backward on
    the GPU, FP32 master weights, Adam).  Parameter order: W0, b0, ..., W3, b3
    with W[l] as [c_out][c_in][3][3]."""

    N_OUT = 15

    def __init__(self, seed=4):
        self._torch = _torch()
        h = ctypes.c_void_p()
        _check(lib().art_cnn_create(int(seed), ctypes.byref(h)))
        self.handle = h
        self.n_params = int(lib().art_cnn_num_params())

    def set_params(self, vec):
        v = np.ascontiguousarray(vec, dtype=np.float32)
        _check(lib().art_cnn_set_params(self.handle, v.ctypes.data, v.size))

    def get_params(self):
        v = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().art_cnn_get_params(self.handle, v.ctypes.data, v.size))
        return v

    def forward(self, x, stream=None):
        """x: CUDA float32 (B, 3, H, W) -> logits (B, 15, H, W)."""
        torch = self._torch
        x = x.contiguous()
        B, C, H, W = x.shape
        assert C == 3 and x.dtype == torch.float32
        z = torch.empty((B, self.N_OUT, H, W), dtype=torch.float32, device=x.device)
        _check(lib().art_cnn_forward(self.handle, x.data_ptr(), B, H, W, z.data_ptr(),
                                     _stream(torch, stream)))
        return z

    def gradients(self, x, labels, valid, pos_weight=1.0, stream=None):
        """(loss, flat gradient) of the batch; labels/valid CUDA uint8 (B, 15, H, W)."""
        torch = self._torch
        x, labels, valid = x.contiguous(), labels.contiguous(), valid.contiguous()
        B, _, H, W = x.shape
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = ctypes.c_float()
        _check(lib().art_cnn_gradients(self.handle, x.data_ptr(), labels.data_ptr(),
                                       valid.data_ptr(), B, H, W, float(pos_weight), g.ctypes.data,
                                       ctypes.byref(loss), _stream(torch, stream)))
        return float(loss.value), g

    def train_step(self, x, labels, valid, lr=1e-3, pos_weight=1.0, want_loss=True, stream=None):
        torch = self._torch
        x, labels, valid = x.contiguous(), labels.contiguous(), valid.contiguous()
        B, _, H, W = x.shape
        loss = ctypes.c_float()
        _check(lib().art_cnn_train_step(self.handle, x.data_ptr(), labels.data_ptr(),
                                        valid.data_ptr(), B, H, W, float(lr), float(pos_weight),
                                        ctypes.byref(loss) if want_loss else None,
                                        _stream(torch, stream)))
        return float(loss.value) if want_loss else None

    def close(self):
        if getattr(self, "handle", None):
            lib().art_cnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cnn_level_shape(cfg, level):
    return ((1 << level) * (int(cfg["ny0"]) - 1) + 1, (1 << level) * (int(cfg["nx0"]) - 1) + 1)


def cnn_features(cfg, img, ft, level, n_abs, stream=None):
    """Network input (1, 3, H, W) float32 of level `level` of a rendered image."""
    torch = _torch()
    H, W = cnn_level_shape(cfg, level)
    x = torch.empty((1, 3, H, W), dtype=torch.float32, device=img.device)
    ny, nx = img.shape[1], img.shape[2]
    _check(lib().art_cnn_features(img.data_ptr(), ft.data_ptr() if ft is not None else None, nx, ny,
                                  int(cfg["nx0"]), int(cfg["ny0"]), int(cfg["levels"]), int(level),
                                  float(n_abs), x.data_ptr(), _stream(torch, stream)))
    return x


def cnn_labels(cfg, lev, level, stream=None):
    """Training labels and valid mask (1, 15, H, W) uint8 from a plain render's level map."""
    torch = _torch()
    H, W = cnn_level_shape(cfg, level)
    lab = torch.empty((1, 15, H, W), dtype=torch.uint8, device=lev.device)
    val = torch.empty((1, 15, H, W), dtype=torch.uint8, device=lev.device)
    ny, nx = lev.shape
    _check(lib().art_cnn_labels(lev.data_ptr(), nx, ny, int(cfg["nx0"]), int(cfg["ny0"]),
                                int(cfg["levels"]), int(level), lab.data_ptr(), val.data_ptr(),
                                _stream(torch, stream)))
    return lab, val
