"""MI355X-native diffuse-radiation ray-tracing sweep (arXiv:1410.0763, Sect. 2.2-3.1)."""
