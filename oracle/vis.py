"""Interferometric visibilities of screen images (test oracle).

Test infrastructure only.  Follows Gelles et al. 2021, Sec. 4.3 (visibility
domain analysis): a visibility is a complex Fourier component of the sky
image, on baseline (u, v) in cycles per unit of screen coordinate,

    V(u, v) = sum_j sum_i  g(x_i) g(y_j) I[j, i] exp(-2 pi i (u x_i + v y_j)) dx^2,

the pixel-sum form of the Fourier integral over the image plane (sign and
normalisation of the standard radio-interferometry convention; V(0, 0) is the
total flux of the tapered image).  Pixel (j, i) sits at the vertex
x_i = (i - (nx-1)/2) dx, y_j = (j - (ny-1)/2) dx of the screen grid, the
image centre on the origin.

Against spurious power from the sharp field edge the paper doubles the field
of view and the pixel number (same pixel size) and applies a Gaussian taper of
FWHM = FOV/4 before the transform; here the taper is

    g(x) = exp(-4 ln 2 x^2 / FWHM^2)   (FWHM <= 0: no taper, g = 1),

applied as the separable product g(x) g(y) of a circular Gaussian.  Reading
(FOV in the FWHM): the field of view before doubling.  The residual
visibilities of the paper are the transform of the residual image (adaptive
minus uniform).
"""
import numpy as np


def axis_coords(n, dx):
    """Pixel-centre coordinates of one image axis, centred on the origin."""
    return (np.arange(n, dtype=np.float64) - 0.5 * (n - 1)) * float(dx)


def taper(n, dx, fwhm):
    """One-axis factor of the circular Gaussian taper of the given FWHM."""
    if fwhm is None or fwhm <= 0:
        return np.ones(n)
    x = axis_coords(n, dx)
    return np.exp(-4.0 * np.log(2.0) * x * x / (float(fwhm) ** 2))


def visibility(img, dx, u, v, fwhm=0.0):
    """V[..., l, k] = V(u_k, v_l) of image planes img[..., ny, nx] (the sum
    over pixels above; the inner sum over x, the outer over y, each a
    matrix product)."""
    img = np.asarray(img, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64).ravel()
    v = np.asarray(v, dtype=np.float64).ravel()
    ny, nx = img.shape[-2:]
    x = axis_coords(nx, dx)
    y = axis_coords(ny, dx)
    gx = taper(nx, dx, fwhm)
    gy = taper(ny, dx, fwhm)
    Ex = np.exp(-2j * np.pi * np.outer(x, u)) * gx[:, None]      # (nx, nu)
    Ey = np.exp(-2j * np.pi * np.outer(v, y)) * gy[None, :]      # (nv, ny)
    return (Ey @ (img @ Ex)) * (float(dx) ** 2)


def visibility_at(img, dx, u, v, fwhm=0.0):
    """V(u, v) at one baseline (a single pixel sum), for sampled checks of
    large images."""
    img = np.asarray(img, dtype=np.float64)
    ny, nx = img.shape[-2:]
    x = axis_coords(nx, dx)
    y = axis_coords(ny, dx)
    ex = np.exp(-2j * np.pi * float(u) * x) * taper(nx, dx, fwhm)
    ey = np.exp(-2j * np.pi * float(v) * y) * taper(ny, dx, fwhm)
    return complex(ey @ (img @ ex)) * float(dx) ** 2


def grid_frequencies(fov, umax):
    """Baselines on the transform grid of a field of view fov, spacing 1/fov,
    |u| <= umax: (u >= 0 half-axis, full axis)."""
    du = 1.0 / float(fov)
    k = int(np.floor(float(umax) / du + 1e-9))
    half = np.arange(0, k + 1) * du
    full = np.arange(-k, k + 1) * du
    return half, full


def doubled_field(cfg):
    """The paper's doubled field: twice the field of view and (2 n0 - 1)
    base points per axis, so the pixel size and level count are unchanged
    and the original grid is the central block of the doubled one."""
    c = dict(cfg)
    c["fov"] = 2.0 * float(cfg["fov"])
    c["nx0"] = 2 * (int(cfg["nx0"]) - 1) + 1
    c["ny0"] = 2 * (int(cfg["ny0"]) - 1) + 1
    return c
