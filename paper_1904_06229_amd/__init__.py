"""MI355X-native exact matrix permanents (Gray-code Glynn/Ryser) behind a C-ABI."""
