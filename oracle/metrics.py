"""FP64 reference of the evaluation metrics -- TEST INFRASTRUCTURE ONLY.

* Eq. 3: scene-linear to sRGB, piecewise with breakpoints 0, 0.0031308 and 1.
* PSNR in sRGB (Sec. 5): peak 1, MSE over all pixels and channels.
* RelMSE (Sec. 5): lambda1 (I_SR - I_HR)^2 / (I_HR^2 + lambda2), averaged over
  all pixels and channels; lambda1 = 0.5, lambda2 = 0.01 on BCR.
* spp_avg = spp_LRHS / s^2 + spp_HRLS for scale s (Sec. 5.1).
"""
import numpy as np


def srgb(l):
    l = np.asarray(l, np.float64)
    out = np.where(l <= 0.0, 0.0,
                   np.where(l <= 0.0031308, 12.92 * l,
                            np.where(l < 1.0, 1.055 * np.power(np.maximum(l, 1e-300), 1 / 2.4) - 0.055,
                                     1.0)))
    return out


def psnr(img, ref):
    mse = np.mean((srgb(img) - srgb(ref)) ** 2)
    return 10.0 * np.log10(1.0 / mse) if mse > 0 else np.inf


def relmse(img, ref, lam1=0.5, lam2=0.01):
    img = np.asarray(img, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.mean(lam1 * (img - ref) ** 2 / (ref ** 2 + lam2)))


def spp_avg(spp_lrhs, spp_hrls, scale):
    return spp_lrhs / scale ** 2 + spp_hrls
