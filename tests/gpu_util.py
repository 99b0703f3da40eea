"""Helpers for the GPU tests: device transfers and error norms (no arithmetic of the method)."""
import numpy as np
import torch


def dev(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_max(got: np.ndarray, ref: np.ndarray) -> float:
    """max |got - ref| / max |ref|."""
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def rel_fro(got: np.ndarray, ref: np.ndarray) -> float:
    return float(np.linalg.norm((got - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))
