"""Training data and training of the learned solver selector."""
