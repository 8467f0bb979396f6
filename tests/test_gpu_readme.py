"""The Python example in README.md runs as written (on one MI355X) and gives a finite gradient."""
import os
import re

import numpy as np
import pytest

README = os.path.join(os.path.dirname(__file__), "..", "README.md")


@pytest.mark.gpu
def test_readme_python_example_runs():
    text = open(README).read()
    blocks = re.findall(r"```python\n(.*?)```", text, flags=re.S)
    assert len(blocks) == 1
    print("[case] README example", flush=True)
    scope = {}
    exec(compile(blocks[0], "README.md", "exec"), scope)
    grad = scope["theta"].grad.numpy()
    assert np.all(np.isfinite(grad)) and np.abs(grad).max() > 0.0
    assert not scope["diverged"].any()
    assert np.isfinite(scope["sums"]).all()
    scope["col"].close()
    scope["batch"].close()
