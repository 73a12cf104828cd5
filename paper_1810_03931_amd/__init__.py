"""MI355X-native ensemble ODE integration (arXiv:1810.03931, Hegedus)."""
