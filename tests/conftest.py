import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu():
    if not gpu_available():
        pytest.skip("no GPU visible")
    import torch
    return torch.device("cuda:0")


def record_error(config: str, precision: str, **metrics) -> None:
    """Appends one JSON line of measured errors to $POLYSPEC_ERROR_LOG (if set) and prints it."""
    import json
    rec = {"config": config, "precision": precision}
    rec.update({k: (float(v) if hasattr(v, "__float__") else v) for k, v in metrics.items()})
    line = json.dumps(rec)
    print(f"[errors] {line}", file=sys.stderr, flush=True)
    path = os.environ.get("POLYSPEC_ERROR_LOG")
    if path:
        with open(path, "a") as fh:
            fh.write(line + "\n")


PRECISION_NAMES = {0: "fp32", 1: "split_bf16", 2: "split_fp16"}
