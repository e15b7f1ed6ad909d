"""Locate (and if absent, build) libsgw.so for the tests."""
import os

from paper_1812_03717_amd import build as _build
from paper_1812_03717_amd import sgw


def ensure_library():
    if not os.path.exists(sgw.LIB_PATH):
        _build.build(verbose=False)
    return sgw.load_library()
