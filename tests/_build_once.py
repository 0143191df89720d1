"""Build the product library and the oracle once per test session if they are
missing (tests load what is built and build only when nothing is)."""
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def ensure_built():
    from paper_2609_29765_amd import build as pb
    from oracle import build as ob
    if not os.path.exists(os.path.join(ROOT, "paper_2609_29765_amd", "libstc.so")):
        pb.build()
    if not os.path.exists(os.path.join(ROOT, "oracle", "liboracle.so")):
        ob.build()
