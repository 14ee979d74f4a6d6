"""Reduced Hessians of the power-flow balance equations on MI355X (librh binding)."""
