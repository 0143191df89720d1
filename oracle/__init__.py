"""Plain serial CPU oracle (test infrastructure only; see oracle.c)."""
