"""Plain CPU reference for JAG filtered search (test infrastructure only)."""
