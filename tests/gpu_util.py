"""Helpers for the GPU tests: host <-> device copies of component planes."""
import numpy as np
import torch


def dev(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy()


def note(*args):
    """Name the case on stdout before a GPU step (flushed)."""
    print("[gpu-case]", *args, flush=True)


def same_bits(a: np.ndarray, b: np.ndarray) -> bool:
    """Bitwise equality treating +0 and -0 as equal (signed zeros compare equal)."""
    return bool(np.array_equal(a, b))
