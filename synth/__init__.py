"""Seeded synthetic inputs (no method arithmetic)."""
