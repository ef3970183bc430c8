"""Test configuration: registers the ``gpu`` marker and puts the repository
root on sys.path so that ``oracle`` and ``paper_0903_1949_amd`` import."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path through the C ABI)")
    config.addinivalue_line("markers", "slow: oracle cases that take tens of seconds on the CPU")
