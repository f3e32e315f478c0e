"""Plain FP64 CPU oracle of the multipatch RK4 wave step (test infrastructure only)."""
