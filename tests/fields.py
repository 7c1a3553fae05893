"""Closed-form test fields shared by the CPU and GPU tests."""
import numpy as np


def square_wave(x, y, H=1.0, terms=8):
    """eq. square of the variable-resolution section: the first `terms`
    terms of the Fourier series of a square wave in x times sin(2 pi y / H),
    with its gradient and Laplacian. Returns (phi, phi_x, phi_y, lap)."""
    phi = np.zeros_like(x)
    px = np.zeros_like(x)
    py = np.zeros_like(x)
    lap = np.zeros_like(x)
    ky = 2.0 * np.pi / H
    sy, cy = np.sin(ky * y), np.cos(ky * y)
    for k in range(1, terms + 1):
        c = 4.0 / (np.pi * (2 * k - 1))
        kx = 2.0 * (2 * k - 1) * np.pi / H
        arg = kx * (x - 0.25 * H)
        sx, cx = np.sin(arg), np.cos(arg)
        phi += c * sy * sx
        px += c * sy * kx * cx
        py += c * ky * cy * sx
        lap -= c * sy * sx * (kx * kx + ky * ky)
    return phi, px, py, lap


def smooth_fields(x, y):
    """Two smooth periodic fields on [0, 2 pi)^2 for operator parity tests."""
    return {"sin_cos": np.sin(x) * np.cos(2 * y),
            "mixed": np.cos(3 * x + y) + 0.3 * np.sin(x - 2 * y) + 2.0}
