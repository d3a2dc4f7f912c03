"""Colour differences between rendered images (analysis of results, not part
of the render): CIE XYZ -> CIELAB and the CIEDE2000 difference (Sharma, Wu
and Dalal, Color Res. Appl. 30 (2005)).  Used to report how far the
surrogate form of bubbly panes is from the exact form."""
import numpy as np


def white_point(cmf, lambda_nm, Y=1.0):
    """XYZ of a flat spectrum under the observer table (trapezoid weights in
    nm, as the render's XYZ), scaled to luminance Y."""
    lam = np.asarray(lambda_nm, dtype=np.float64)
    cmf = np.asarray(cmf, dtype=np.float64).reshape(-1, 3)
    if len(lam) == 1:
        w = np.ones(1)
    else:
        w = np.empty(len(lam))
        w[1:-1] = 0.5 * (lam[2:] - lam[:-2])
        w[0] = 0.5 * (lam[1] - lam[0])
        w[-1] = 0.5 * (lam[-1] - lam[-2])
    xyz = (w[:, None] * cmf).sum(0)
    return xyz * (Y / xyz[1])


def xyz_to_lab(xyz, white):
    xyz = np.asarray(xyz, dtype=np.float64)
    t = xyz / np.asarray(white, dtype=np.float64)
    d = 6.0 / 29.0
    f = np.where(t > d ** 3, np.cbrt(np.maximum(t, 0.0)), t / (3 * d * d) + 4.0 / 29.0)
    L = 116.0 * f[..., 1] - 16.0
    a = 500.0 * (f[..., 0] - f[..., 1])
    b = 200.0 * (f[..., 1] - f[..., 2])
    return np.stack([L, a, b], -1)


def delta_e2000(lab1, lab2):
    lab1 = np.asarray(lab1, dtype=np.float64)
    lab2 = np.asarray(lab2, dtype=np.float64)
    L1, a1, b1 = lab1[..., 0], lab1[..., 1], lab1[..., 2]
    L2, a2, b2 = lab2[..., 0], lab2[..., 1], lab2[..., 2]
    C1, C2 = np.hypot(a1, b1), np.hypot(a2, b2)
    Cm = 0.5 * (C1 + C2)
    G = 0.5 * (1.0 - np.sqrt(Cm ** 7 / (Cm ** 7 + 25.0 ** 7)))
    a1p, a2p = (1 + G) * a1, (1 + G) * a2
    C1p, C2p = np.hypot(a1p, b1), np.hypot(a2p, b2)
    h1p = np.degrees(np.arctan2(b1, a1p)) % 360.0
    h2p = np.degrees(np.arctan2(b2, a2p)) % 360.0
    dLp = L2 - L1
    dCp = C2p - C1p
    prod = C1p * C2p
    dh = h2p - h1p
    dh = np.where(dh > 180.0, dh - 360.0, np.where(dh < -180.0, dh + 360.0, dh))
    dh = np.where(prod == 0.0, 0.0, dh)
    dHp = 2.0 * np.sqrt(prod) * np.sin(np.radians(dh) / 2.0)
    Lpm = 0.5 * (L1 + L2)
    Cpm = 0.5 * (C1p + C2p)
    hs = h1p + h2p
    hpm = np.where(np.abs(h1p - h2p) <= 180.0, hs / 2.0,
                   np.where(hs < 360.0, (hs + 360.0) / 2.0, (hs - 360.0) / 2.0))
    hpm = np.where(prod == 0.0, hs, hpm)
    T = (1 - 0.17 * np.cos(np.radians(hpm - 30)) + 0.24 * np.cos(np.radians(2 * hpm))
         + 0.32 * np.cos(np.radians(3 * hpm + 6)) - 0.20 * np.cos(np.radians(4 * hpm - 63)))
    dtheta = 30.0 * np.exp(-((hpm - 275.0) / 25.0) ** 2)
    RC = 2.0 * np.sqrt(Cpm ** 7 / (Cpm ** 7 + 25.0 ** 7))
    SL = 1 + 0.015 * (Lpm - 50) ** 2 / np.sqrt(20 + (Lpm - 50) ** 2)
    SC = 1 + 0.045 * Cpm
    SH = 1 + 0.015 * Cpm * T
    RT = -np.sin(np.radians(2 * dtheta)) * RC
    return np.sqrt((dLp / SL) ** 2 + (dCp / SC) ** 2 + (dHp / SH) ** 2 + RT * (dCp / SC) * (dHp / SH))


def image_delta_e(xyz_a, xyz_b, cmf, lambda_nm, percentile=99.0):
    """Per-pixel CIEDE2000 between two XYZ images; the white is a flat
    spectrum at the given percentile of image A's luminance."""
    Y = float(np.percentile(np.asarray(xyz_a)[..., 1], percentile))
    wp = white_point(cmf, lambda_nm, Y if Y > 0 else 1.0)
    return delta_e2000(xyz_to_lab(xyz_a, wp), xyz_to_lab(xyz_b, wp))
