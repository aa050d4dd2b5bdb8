"""Regenerate the device headers and JSON tables: python -m paper_2102_08518_amd.gen"""
import sys

from .emit import generate

if __name__ == "__main__":
    generate(sys.argv[1:] or None)
