"""The binding and PyTorch share one HIP runtime in the process."""
import os


def test_single_hip_runtime_loaded():
    import paper_2505_18681_amd  # noqa: F401
    import torch  # noqa: F401

    with open(f"/proc/{os.getpid()}/maps") as f:
        libs = {line.split()[-1] for line in f if "libamdhip64" in line}
    assert len(libs) == 1, f"more than one HIP runtime mapped: {sorted(libs)}"
