"""MI355X-native ADER-DG step with the a-posteriori subcell (MOOD) limiter."""
