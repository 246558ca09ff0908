"""Solver metrics of Sec. 5.2 on the device: the angle between each estimated
vector and its reference, and the eigenvector streak (the number of leading
estimates each within eps of its reference, counted until the first miss).
The float64 Grams come from the library's Gram kernel; only the k cosines
travel to the host."""
from __future__ import annotations

import math

import numpy as np
import torch

from . import sped


def vector_angles(Vref: torch.Tensor, V: torch.Tensor) -> np.ndarray:
    """Sign-free angle between column i of Vref and column i of V."""
    if Vref.shape != V.shape:
        raise ValueError("blocks differ in shape")
    V = V.to(Vref.dtype)
    c = sped.gram(Vref, V).diagonal().cpu().numpy()
    na = sped.gram(Vref).diagonal().cpu().numpy()
    nb = sped.gram(V).diagonal().cpu().numpy()
    cos = np.abs(c) / np.sqrt(na * nb)
    return np.arccos(np.clip(cos, 0.0, 1.0))


def eigenvector_streak(Vref: torch.Tensor, V: torch.Tensor, eps: float = math.pi / 8) -> int:
    streak = 0
    for a in vector_angles(Vref, V):
        if a > eps:
            break
        streak += 1
    return streak
