"""The library and torch share one HIP runtime whatever the import order."""
import subprocess
import sys

import pytest

SNIPPET = """
import paper_2509_17340_amd
maps = open('/proc/self/maps').read().split('\\n')
paths = sorted({l.split()[-1] for l in maps if 'libamdhip64' in l or 'libhsa-runtime64' in l})
print('\\n'.join(paths))
"""


@pytest.mark.skipif(not sys.platform.startswith("linux"), reason="reads /proc/self/maps")
def test_one_hip_runtime_when_the_package_is_imported_first():
    out = subprocess.run([sys.executable, "-c", SNIPPET], capture_output=True, text=True,
                         timeout=300, cwd=__file__.rsplit("/tests/", 1)[0])
    assert out.returncode == 0, out.stderr
    paths = out.stdout.split()
    hip = [p for p in paths if "libamdhip64" in p]
    hsa = [p for p in paths if "libhsa-runtime64" in p]
    assert len(hip) == 1 and len(hsa) == 1, paths
