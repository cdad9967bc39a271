"""Plain CPU reference for the shifted Hessenberg solves (test infrastructure only)."""
